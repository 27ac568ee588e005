// Internal declarations of the LDG library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ldg.h"

namespace ldg {

constexpr int TILE = 64;   // elements per tile of the element-fastest layouts
constexpr int NSLOT = 5;   // stored D-dependent blocks per element: B^1, B^2, U_0, U_1, U_2

// ---- element-fastest ("tiled") layouts ------------------------------------
// vectors:  (k, i)    -> [k/64][i][k%64]
// blocks :  (k, s, f) -> [k/64][s][f/2][k%64][f%2],  f = i*N + j, pairs of doubles
__host__ __device__ inline int64_t vidx(int64_t k, int i, int N) {
  return (k >> 6) * (int64_t)(TILE * N) + (int64_t)i * TILE + (k & 63);
}
__host__ __device__ constexpr int npairs(int N) { return (N * N + 1) / 2; }
// Gauss points per edge of the edge-trace form of the neighbour blocks: the
// integrands d phi_i phi_j of the off-diagonal edge terms have degree 3p on
// the edge, so ceil((3p + 1) / 2) points integrate them exactly
__host__ __device__ constexpr int edge_trace_points(int N) {
  int p = 0;
  while ((p + 1) * (p + 2) / 2 < N) ++p;
  return (3 * p + 2) / 2;
}
// The volume term sum_m G^m Z^m of the same apply as a quadrature: the
// integrand dphi_i/dx_m d_h Z_h has degree D = 3p - 1.  The unit square
// collapsed onto the triangle (x1 = u, x2 = (1 - u) v, Jacobian 1 - u) with
// Gauss-Jacobi points for the weight 1 - u in u and Gauss-Legendre points in v
// integrates it exactly with ceil((D + 1) / 2) points in each; none at p = 0,
// where the term vanishes
__host__ __device__ constexpr int vol_points_u(int N) {
  int p = 0;
  while ((p + 1) * (p + 2) / 2 < N) ++p;
  return p == 0 ? 0 : (3 * p - 1 + 2) / 2;
}
__host__ __device__ constexpr int vol_points_v(int N) {
  int p = 0;
  while ((p + 1) * (p + 2) / 2 < N) ++p;
  return p == 0 ? 0 : (3 * p - 1 + 2) / 2;
}
__host__ __device__ constexpr int vol_points(int N) { return vol_points_u(N) * vol_points_v(N); }
// rows (coefficient index l) of the FP64 / FP32 A-operand tables of the MFMA
// block assembly: its k-steps of four cover l < 4 ceil(N / 4); 16 rows for
// N <= 15, 24 for N = 21, 28 for N = 28
__host__ __device__ constexpr int mfma_lrows(int N) { return N <= 16 ? 16 : (N + 3) / 4 * 4; }
__host__ __device__ inline int64_t pidx(int64_t k, int s, int pr, int ns, int np) {
  return ((((k >> 6) * ns + s) * (int64_t)np + pr) * TILE + (k & 63)) * 2;
}

// ---- geometry in structure-of-arrays form, n-major per local edge --------
struct Geo {
  int64_t K, Kpad;
  const double* area2;   // [Kpad]      2|T_k| = det B_k
  const double* B;       // [4][Kpad]   B11, B12, B21, B22
  const double* a1;      // [2][Kpad]   first vertex
  const double* elen;    // [3][Kpad]   |E_kn|
  const double* nu;      // [3][2][Kpad] exterior unit normal (n, m)
  const int32_t* nbr;    // [3][Kpad]   k+ or -1
  const int8_t* nbrn;    // [3][Kpad]   n+
  const int8_t* kind;    // [3][Kpad]   ldg_edge_kind
  const int32_t* bidx;   // [3][Kpad]   boundary edge index or -1
  // FP32 copies for the FP32 apply kernels: the values those kernels would
  // round the FP64 ones to (so the results are the same bits), in half the bytes
  const float* ainv32;   // [Kpad]      -1 / (2|T_k|)
  const float* B32;      // [4][Kpad]
  const float* elen32;   // [3][Kpad]
  const float* nu32;     // [3][2][Kpad]
};

// ---- reference data computed on the host --------------------------------
struct RefData {
  int p = 0, N = 1, NN = 1;
  // 2D matrices, row-major [i][j]
  std::vector<double> M, H[2], Sd[3], So[3][3];
  // 3-index tensors stored [l][i][j]
  std::vector<double> G[2], Rd[3], Ro[3][3];
  // projection rule (order max(2p,1)) and boundary rule (order 2p+1)
  std::vector<double> q1, q2, w, s, ws;
  int R = 0, R1 = 0;
};

// host_ref.cpp
int num_basis(int p);
double phi_hat(int i, double x1, double x2);
double dphi_hat(int i, int m, double x1, double x2);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);  // on (0,1)
void gauss_jacobi10(int n, std::vector<double>& x, std::vector<double>& w);  // on (0,1), weight 1-u
void projection_rule(int p, std::vector<double>& q1, std::vector<double>& q2,
                     std::vector<double>& w);
RefData build_refdata(int p, int policy);   // policy: ldg_quad_policy

// host_mesh.cpp
struct HostMesh {
  int64_t K = 0, Kpad = 0;
  std::vector<double> area2, B, a1, elen, nu;
  std::vector<int32_t> nbr, bidx;
  std::vector<int8_t> nbrn, kind;
  std::vector<int32_t> bedge_k;  // boundary edges: triangle
  std::vector<int8_t> bedge_n;   //                 local edge
  std::vector<int32_t> belem;    // triangles with at least one boundary edge
  int64_t E_int = 0;
};
// returns "" on success, else the error text; *is_mesh_error distinguishes EMESH from EINVAL
std::string build_mesh(const double* coordV, int64_t numV, const int32_t* V0T, int64_t K,
                       const int8_t* edge_kind, HostMesh& out, bool* is_mesh_error);

// host_io.cpp: MEDIT mesh reader and VTK unstructured-grid writer; "" on success
std::string read_medit(const char* path, std::vector<double>& coordV, std::vector<int32_t>& V0T,
                       std::vector<int32_t>& edge_id);
std::string write_vtu(const char* path, const char* name, const std::vector<double>& coordV,
                      const std::vector<int32_t>& V0T, int64_t K, int nL, const double* lagr,
                      bool binary);

}  // namespace ldg
