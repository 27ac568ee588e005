// Mesh input and VTK output on the host.
//
// Reader: the ASCII MEDIT ".mesh" format that Gmsh writes (sections
// "Vertices", "Edges", "Triangles"; 1-based vertex numbers, a reference
// number per entity), as the paper's circle-domain generator reads it
// (Sec. 4, domainCircle): vertex coordinates, triangles, and the boundary ID
// of every boundary edge listed in "Edges".
//
// Writer: an XML VTK unstructured-grid file of a discontinuous piecewise
// polynomial given by its values at the Lagrange points of every triangle
// (Sec. 3.8): each triangle carries its own points, as a linear triangle
// (3 values) or a quadratic one (6 values).
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "ldg_internal.h"

namespace ldg {

namespace {

uint64_t edge_key(int64_t a, int64_t b) {
  if (a > b) std::swap(a, b);
  return ((uint64_t)a << 32) | (uint64_t)b;
}

bool next_token(std::istream& in, std::string& tok) {
  while (in >> tok) {
    if (tok[0] == '#') {   // comment to the end of the line
      std::string rest;
      std::getline(in, rest);
      continue;
    }
    return true;
  }
  return false;
}

bool read_int(std::istream& in, int64_t* v) {
  std::string t;
  if (!next_token(in, t)) return false;
  char* end = nullptr;
  errno = 0;
  const long long x = std::strtoll(t.c_str(), &end, 10);
  if (errno || *end) return false;
  *v = x;
  return true;
}

bool read_real(std::istream& in, double* v) {
  std::string t;
  if (!next_token(in, t)) return false;
  char* end = nullptr;
  errno = 0;
  *v = std::strtod(t.c_str(), &end);
  return !errno && !*end && std::isfinite(*v);
}

const char B64[] = "ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/";

void base64_append(std::string& out, const unsigned char* p, size_t n) {
  size_t i = 0;
  for (; i + 3 <= n; i += 3) {
    const uint32_t v = (uint32_t)p[i] << 16 | (uint32_t)p[i + 1] << 8 | p[i + 2];
    out += B64[v >> 18];
    out += B64[(v >> 12) & 63];
    out += B64[(v >> 6) & 63];
    out += B64[v & 63];
  }
  if (i < n) {
    uint32_t v = (uint32_t)p[i] << 16;
    if (i + 1 < n) v |= (uint32_t)p[i + 1] << 8;
    out += B64[v >> 18];
    out += B64[(v >> 12) & 63];
    out += i + 1 < n ? B64[(v >> 6) & 63] : '=';
    out += '=';
  }
}

// VTK XML "binary" data: base64 of a UInt32 byte count followed by the bytes
template <class T>
std::string vtk_binary(const std::vector<T>& v) {
  const uint32_t nb = (uint32_t)(v.size() * sizeof(T));
  std::vector<unsigned char> buf(sizeof(uint32_t) + nb);
  std::memcpy(buf.data(), &nb, sizeof(uint32_t));
  if (nb) std::memcpy(buf.data() + sizeof(uint32_t), v.data(), nb);
  std::string s;
  s.reserve(buf.size() * 4 / 3 + 8);
  base64_append(s, buf.data(), buf.size());
  return s;
}

template <class T>
void vtk_array(std::ostream& o, const char* type, const char* name, int ncomp,
               const std::vector<T>& v, bool binary, const char* fmt) {
  o << "        <DataArray type=\"" << type << "\"";
  if (name) o << " Name=\"" << name << "\"";
  if (ncomp > 1) o << " NumberOfComponents=\"" << ncomp << "\"";
  o << " format=\"" << (binary ? "binary" : "ascii") << "\">\n";
  if (binary) {
    o << "          " << vtk_binary(v) << "\n";
  } else {
    char buf[64];
    for (size_t i = 0; i < v.size(); ++i) {
      std::snprintf(buf, sizeof(buf), fmt, v[i]);
      o << (i % ncomp == 0 ? "          " : " ") << buf << (i % ncomp == (size_t)ncomp - 1 ? "\n" : "");
    }
  }
  o << "        </DataArray>\n";
}

}  // namespace

std::string read_medit(const char* path, std::vector<double>& coordV, std::vector<int32_t>& V0T,
                       std::vector<int32_t>& edge_id) {
  std::ifstream in(path);
  if (!in) return std::string("cannot open ") + path;
  int64_t numV = -1, K = -1, dim = 3;   // Gmsh writes "Dimension 3": x y z ref per vertex
  std::vector<int64_t> bed;   // boundary edges: v1, v2, id (0-based vertices)
  std::string tok;
  while (next_token(in, tok)) {
    if (tok == "Dimension") {
      if (!read_int(in, &dim) || (dim != 2 && dim != 3)) return "bad dimension";
    } else if (tok == "Vertices") {
      if (!read_int(in, &numV) || numV < 3 || numV > (int64_t)1 << 31)
        return "bad vertex count";
      coordV.assign(2 * numV, 0.0);
      for (int64_t v = 0; v < numV; ++v) {
        double x[3];
        int64_t ref;
        for (int d = 0; d < dim; ++d)
          if (!read_real(in, &x[d])) return "bad vertex line";
        if (!read_int(in, &ref)) return "bad vertex line";
        coordV[2 * v] = x[0];
        coordV[2 * v + 1] = x[1];
      }
    } else if (tok == "Edges") {
      int64_t ne;
      if (!read_int(in, &ne) || ne < 0) return "bad edge count";
      bed.resize(3 * ne);
      for (int64_t e = 0; e < ne; ++e) {
        int64_t a, b, id;
        if (!read_int(in, &a) || !read_int(in, &b) || !read_int(in, &id)) return "bad edge line";
        bed[3 * e] = a - 1;
        bed[3 * e + 1] = b - 1;
        bed[3 * e + 2] = id;
      }
    } else if (tok == "Triangles") {
      if (!read_int(in, &K) || K < 1 || K > (int64_t)1 << 30) return "bad triangle count";
      V0T.assign(3 * K, 0);
      for (int64_t k = 0; k < K; ++k) {
        int64_t a, b, c, ref;
        if (!read_int(in, &a) || !read_int(in, &b) || !read_int(in, &c) || !read_int(in, &ref))
          return "bad triangle line";
        V0T[3 * k] = (int32_t)(a - 1);
        V0T[3 * k + 1] = (int32_t)(b - 1);
        V0T[3 * k + 2] = (int32_t)(c - 1);
      }
    } else if (tok == "End") {
      break;
    }
  }
  if (numV < 0 || K < 0) return "no Vertices or no Triangles section";
  for (int64_t k = 0; k < 3 * K; ++k)
    if (V0T[k] < 0 || V0T[k] >= numV) return "triangle vertex out of range";
  for (size_t e = 0; e < bed.size(); e += 3)
    if (bed[e] < 0 || bed[e] >= numV || bed[e + 1] < 0 || bed[e + 1] >= numV)
      return "edge vertex out of range";
  // counter-clockwise order (the orientation the method assumes, Sec. 3.2)
  for (int64_t k = 0; k < K; ++k) {
    const double* a = &coordV[2 * (int64_t)V0T[3 * k]];
    const double* b = &coordV[2 * (int64_t)V0T[3 * k + 1]];
    const double* c = &coordV[2 * (int64_t)V0T[3 * k + 2]];
    const double det = (b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]);
    if (det < 0.0) std::swap(V0T[3 * k + 1], V0T[3 * k + 2]);
  }
  // local edge n joins local vertices n+1 and n+2: 0 if shared by two
  // triangles, else the listed boundary ID, else -1
  std::unordered_map<uint64_t, int> count;
  count.reserve(3 * K);
  for (int64_t k = 0; k < K; ++k)
    for (int n = 0; n < 3; ++n)
      ++count[edge_key(V0T[3 * k + (n + 1) % 3], V0T[3 * k + (n + 2) % 3])];
  std::unordered_map<uint64_t, int64_t> ids;
  for (size_t e = 0; e < bed.size(); e += 3) ids[edge_key(bed[e], bed[e + 1])] = bed[e + 2];
  edge_id.assign(3 * K, 0);
  for (int64_t k = 0; k < K; ++k)
    for (int n = 0; n < 3; ++n) {
      const uint64_t key = edge_key(V0T[3 * k + (n + 1) % 3], V0T[3 * k + (n + 2) % 3]);
      const int cnt = count[key];
      if (cnt > 2) return "an edge is shared by more than two triangles";
      if (cnt == 2) continue;
      auto it = ids.find(key);
      if (it != ids.end() && it->second <= 0) return "a boundary edge has an ID <= 0";
      edge_id[3 * k + n] = it == ids.end() ? -1 : (int32_t)it->second;
    }
  return "";
}

std::string write_vtu(const char* path, const char* name, const std::vector<double>& coordV,
                      const std::vector<int32_t>& V0T, int64_t K, int nL, const double* lagr,
                      bool binary) {
  if (nL != 1 && nL != 3 && nL != 6) return "Lagrange values per triangle must be 1, 3 or 6";
  const int np = nL == 6 ? 6 : 3;
  std::vector<float> pts((size_t)3 * np * K), val((size_t)np * K);
  std::vector<int32_t> conn((size_t)np * K), offs(K);
  std::vector<uint8_t> types(K, nL == 6 ? 22 : 5);   // quadratic / linear triangle
  // Lagrange values come as vertices 1, 2, 3 then the midpoints of the edges
  // opposite vertices 1, 2, 3; the quadratic cell lists the midpoints of
  // (v1, v2), (v2, v3), (v3, v1)
  const int perm[6] = {0, 1, 2, 5, 3, 4};
  for (int64_t k = 0; k < K; ++k) {
    double x[6], y[6];
    for (int i = 0; i < 3; ++i) {
      x[i] = coordV[2 * (int64_t)V0T[3 * k + i]];
      y[i] = coordV[2 * (int64_t)V0T[3 * k + i] + 1];
    }
    for (int i = 0; i < 3; ++i) {   // midpoint of (v_i, v_{i+1})
      x[3 + i] = 0.5 * (x[i] + x[(i + 1) % 3]);
      y[3 + i] = 0.5 * (y[i] + y[(i + 1) % 3]);
    }
    for (int q = 0; q < np; ++q) {
      const size_t pi = (size_t)np * k + q;
      pts[3 * pi] = (float)x[q];
      pts[3 * pi + 1] = (float)y[q];
      pts[3 * pi + 2] = 0.0f;
      conn[pi] = (int32_t)pi;
      val[pi] = (float)(nL == 1 ? lagr[k] : lagr[(size_t)nL * k + (nL == 6 ? perm[q] : q)]);
    }
    offs[k] = (int32_t)(np * (k + 1));
  }
  std::ofstream o(path, std::ios::binary);
  if (!o) return std::string("cannot write ") + path;
  o << "<?xml version=\"1.0\"?>\n"
    << "<VTKFile type=\"UnstructuredGrid\" version=\"0.1\" byte_order=\"LittleEndian\""
    << " header_type=\"UInt32\">\n"
    << "  <UnstructuredGrid>\n"
    << "    <Piece NumberOfPoints=\"" << np * K << "\" NumberOfCells=\"" << K << "\">\n"
    << "      <Points>\n";
  vtk_array(o, "Float32", nullptr, 3, pts, binary, "%.9g");
  o << "      </Points>\n      <Cells>\n";
  vtk_array(o, "Int32", "connectivity", 1, conn, binary, "%d");
  vtk_array(o, "Int32", "offsets", 1, offs, binary, "%d");
  std::vector<int32_t> types32(types.begin(), types.end());
  if (binary) {
    vtk_array(o, "UInt8", "types", 1, types, true, "%d");
  } else {
    vtk_array(o, "UInt8", "types", 1, types32, false, "%d");
  }
  o << "      </Cells>\n      <PointData Scalars=\"" << name << "\">\n";
  vtk_array(o, "Float32", name, 1, val, binary, "%.9g");
  o << "      </PointData>\n    </Piece>\n  </UnstructuredGrid>\n</VTKFile>\n";
  o.close();
  if (!o) return std::string("error writing ") + path;
  return "";
}

}  // namespace ldg
