// Grid lists of Table 1 (Sec. 3.1) on the host, in structure-of-arrays form.
#include <cmath>
#include <unordered_map>

#include "ldg_internal.h"

namespace ldg {

std::string build_mesh(const double* coordV, int64_t numV, const int32_t* V0T, int64_t K,
                       const int8_t* edge_kind, HostMesh& m, bool* is_mesh_error) {
  *is_mesh_error = false;
  if (K <= 0 || numV < 3) return "empty mesh";
  if (K > (int64_t)1 << 30) return "too many triangles";
  for (int64_t k = 0; k < 3 * K; ++k)
    if (V0T[k] < 0 || V0T[k] >= numV) return "vertex index out of range";
  for (int64_t k = 0; k < 3 * K; ++k)
    if (edge_kind[k] < LDG_EDGE_INTERIOR || edge_kind[k] > LDG_EDGE_NEUMANN)
      return "edge kind out of range";
  const int64_t Kp = (K + TILE - 1) / TILE * TILE;
  m.K = K;
  m.Kpad = Kp;
  m.area2.assign(Kp, 1.0);
  m.B.assign(4 * Kp, 0.0);
  m.a1.assign(2 * Kp, 0.0);
  m.elen.assign(3 * Kp, 0.0);
  m.nu.assign(6 * Kp, 0.0);
  m.nbr.assign(3 * Kp, -1);
  m.bidx.assign(3 * Kp, -1);
  m.nbrn.assign(3 * Kp, 0);
  m.kind.assign(3 * Kp, LDG_EDGE_DIRICHLET);
  *is_mesh_error = true;
  for (int64_t k = 0; k < K; ++k) {
    const double* a = coordV + 2 * (int64_t)V0T[3 * k];
    const double* b = coordV + 2 * (int64_t)V0T[3 * k + 1];
    const double* c = coordV + 2 * (int64_t)V0T[3 * k + 2];
    // B_k = [a2 - a1 | a3 - a1] (eq:affinemappings:Fk)
    const double B11 = b[0] - a[0], B12 = c[0] - a[0];
    const double B21 = b[1] - a[1], B22 = c[1] - a[1];
    const double det = B11 * B22 - B12 * B21;
    if (!(det > 0.0)) return "triangle " + std::to_string(k) + " is not counter-clockwise";
    m.area2[k] = det;
    m.B[k] = B11; m.B[Kp + k] = B12; m.B[2 * Kp + k] = B21; m.B[3 * Kp + k] = B22;
    m.a1[k] = a[0]; m.a1[Kp + k] = a[1];
    for (int n = 0; n < 3; ++n) {
      const double* s = coordV + 2 * (int64_t)V0T[3 * k + (n + 1) % 3];
      const double* e = coordV + 2 * (int64_t)V0T[3 * k + (n + 2) % 3];
      const double ex = e[0] - s[0], ey = e[1] - s[1];
      const double L = std::sqrt(ex * ex + ey * ey);
      m.elen[n * Kp + k] = L;
      m.nu[(n * 2 + 0) * Kp + k] = ey / L;     // direction rotated by -pi/2
      m.nu[(n * 2 + 1) * Kp + k] = -ex / L;
    }
  }
  std::unordered_map<uint64_t, int64_t> first;
  first.reserve((size_t)(2 * K));
  int64_t nint = 0;
  for (int64_t k = 0; k < K; ++k)
    for (int n = 0; n < 3; ++n) {
      const uint64_t vs = (uint32_t)V0T[3 * k + (n + 1) % 3];
      const uint64_t ve = (uint32_t)V0T[3 * k + (n + 2) % 3];
      if (vs == ve) return "degenerate edge";
      const uint64_t key = vs < ve ? (vs << 32) | ve : (ve << 32) | vs;
      auto it = first.find(key);
      if (it == first.end()) {
        first.emplace(key, 3 * k + n);
        continue;
      }
      if (it->second < 0) return "edge shared by more than two triangles";
      const int64_t k2 = it->second / 3;
      const int n2 = (int)(it->second % 3);
      if ((uint64_t)V0T[3 * k2 + (n2 + 1) % 3] != ve)
        return "neighbouring triangles traverse a shared edge in the same direction";
      m.nbr[n * Kp + k] = (int32_t)k2;
      m.nbrn[n * Kp + k] = (int8_t)n2;
      m.nbr[n2 * Kp + k2] = (int32_t)k;
      m.nbrn[n2 * Kp + k2] = (int8_t)n;
      it->second = -1;
      ++nint;
    }
  m.E_int = nint;
  m.bedge_k.clear();
  m.bedge_n.clear();
  m.belem.clear();
  for (int64_t k = 0; k < K; ++k) {
    bool has_bnd = false;
    for (int n = 0; n < 3; ++n) {
      const int kind = edge_kind[3 * k + n];
      const bool interior = m.nbr[n * Kp + k] >= 0;
      if (interior != (kind == LDG_EDGE_INTERIOR))
        return "edge kind of triangle " + std::to_string(k) + " edge " + std::to_string(n) +
               " disagrees with the topology";
      m.kind[n * Kp + k] = (int8_t)kind;
      if (!interior) {
        m.bidx[n * Kp + k] = (int32_t)m.bedge_k.size();
        m.bedge_k.push_back((int32_t)k);
        m.bedge_n.push_back((int8_t)n);
        has_bnd = true;
      }
    }
    if (has_bnd) m.belem.push_back((int32_t)k);
  }
  *is_mesh_error = false;
  return "";
}

}  // namespace ldg
