// HBM-resident batched dense kernels for blocks too large for the on-chip
// factor kernels: the node-layer blocks of large subdomains (3-d cells of 16^3
// elements give blocks of 3 * 17^2 = 867 unknowns) and the dense coarse
// matrix.
//
// Matrices are stored as 64 x 64 tiles. A symmetric matrix of order n keeps
// its lower tiles (I >= J, diagonal tiles in full) of the matrix padded to
// 64 * ntb rows, tile index I (I + 1) / 2 + J. Inside a tile two layouts are
// used, both in units of the matrix cores' 16 x 16 x 4 FP64 operation:
//   C layout (accumulators): element (r, c) of a tile at
//     ((r / 16 * 4 + c / 16) * 4 + r % 16 / 4) * 64 + (r % 4) * 16 + c % 16,
//     so each 64-element run is one accumulator register of one wave;
//   A layout (operands): element (r, c) at
//     (r / 16 * 16 + c / 4) * 64 + (c % 4) * 16 + r % 16,
//     so each 64-element run is one operand fragment (lane = row % 16 +
//     16 * (column % 4)).
#pragma once

#include "tpcg_internal.h"

namespace tpcg {

constexpr int kBT = 64;                // tile edge
constexpr int kBTE = kBT * kBT;        // elements per tile

__host__ __device__ inline int big_ntb(int n) { return (n + kBT - 1) / kBT; }
__host__ __device__ inline int big_nl(int ntb) { return ntb * (ntb + 1) / 2; }
__host__ __device__ inline int big_ltile(int I, int J) { return I * (I + 1) / 2 + J; }
__host__ __device__ inline int big_cofs(int r, int c) {
  return ((((r >> 4) * 4 + (c >> 4)) * 4 + ((r & 15) >> 2)) << 6) + ((r & 3) << 4) + (c & 15);
}
__host__ __device__ inline int big_aofs(int r, int c) {
  return (((r >> 4) * 16 + (c >> 2)) << 6) + ((c & 3) << 4) + (r & 15);
}

// Whether the subdomain blocks of g take the HBM-resident path: blocks larger
// than the on-chip kernels take, of odd size, element layers wider than a
// wave, or forced by the problem (big_min_nb).
bool local_is_big(const Geometry& g, int big_min_nb);
// nullptr when the HBM-resident kernels take geometry g, else the reason
const char* big_limits(const Geometry& g);

// Workspace (doubles) of the batched sweep inversion of nmat matrices of
// ntb x ntb tiles, beside the matrices themselves: the pivot inverses and
// the two panels of a step.
inline size_t sweep_ws_elems(int nmat, int ntb) {
  return (size_t)nmat * kBTE * (1 + 2 * (size_t)ntb);
}

// In-place inversion of nmat symmetric positive definite matrices (lower
// tiles, C layout, nl = big_nl(ntb) tiles per matrix at stride mstride
// elements) by the symmetric block sweep; on exit each matrix holds -A^-1.
// flag[0] = 1 on a non-positive pivot. ws: sweep_ws_elems(nmat, ntb).
void sweep_invert(double* S, size_t mstride, int nmat, int ntb, double* ws, int* flag,
                  hipStream_t st);
// The same sweep over the pivots of the first npiv tiles only (the
// remaining tiles receive the Schur complement and the multipliers).
void sweep_pivots(double* S, size_t mstride, int nmat, int ntb, int npiv, double* ws, int* flag,
                  hipStream_t st);

// Coarse matrix as an HBM-resident block-tridiagonal LDL^T factorisation:
// per system, row-major nbc x nbc blocks S_b^-1 [nblkc], L_{b,b-1} [nblkc]
// (block 0 unused) and L_{b+1,b}^T [nblkc] (the last unused). From the
// block-tridiagonal assembly Ac [nsys][nblkc][2][nbc][nbc].
inline size_t coarse_band_elems(const Geometry& g) { return 3 * (size_t)g.nblkc * g.nbc * g.nbc; }
inline size_t coarse_band_ws_elems(const Geometry& g, int nsys) {
  const int ntb2 = 2 * big_ntb(g.nbc);
  return (size_t)nsys * big_nl(ntb2) * kBTE + sweep_ws_elems(nsys, ntb2);
}
void coarse_band_factor(const Geometry& g, const double* Ac, size_t astride, int nsys,
                        double* cband, double* ws, int* flag, hipStream_t st);
// x_c = K_c^-1 y_c for every running system ([nsys][nt]): the forward chain
// into cw ([nsys][nt]), the block-diagonal solve, the backward chain.
void coarse_band_solve(const Geometry& g, const double* cband, const double* yc, double* xc,
                       double* cw, int nsys, const Gate& gate, hipStream_t st);

// Dense coarse path: K_c from its block-tridiagonal assembly (Ac [nsys][nblkc][2][nbc][nbc])
// into lower tiles, the sweep, and the lower tiles of K_c^-1 (row-major, zero past nt) into cpk.
void coarse_dense_inverse(const Geometry& g, const double* Ac, size_t astride, int nsys,
                          double* S, double* ws, double* cpk, int* flag, hipStream_t st);
inline size_t coarse_dense_ws_elems(const Geometry& g, int nsys) {
  const int ntb = big_ntb(g.nt);
  const size_t sweep = (size_t)nsys * big_nl(ntb) * kBTE + sweep_ws_elems(nsys, ntb);
  const size_t dense = (size_t)nsys * g.nt * g.nt;   // the block-tridiagonal path's inverse
  return sweep > dense ? sweep : dense;
}
// Lower tiles of a dense row-major K_c^-1 [nsys][nt][nt] into cpk.
void coarse_pack_inverse(const Geometry& g, const double* inv, int nsys, double* cpk,
                         hipStream_t st);
// Whether the coarse matrix's blocks fit the on-chip block-tridiagonal
// factor and inverse kernels (their column-chunk inverse spreads over the
// chip; the sweep's 64 x 64 pivots are latency-bound at these sizes).
inline bool coarse_btri_fits(const Geometry& g) {
  return g.nbc <= 96 && (g.nbc & 1) == 0;
}

// Sizes of the HBM-resident local factors of geometry g.
struct BigShape {
  int ntb, nl, npad;
  size_t rec_dir;   // elements of one Dirichlet record (lower tiles)
  size_t rec_neu;   // elements of one Neumann record (all tiles)
};
__host__ __device__ inline BigShape big_shape(const Geometry& g) {
  BigShape b;
  b.ntb = big_ntb(g.nb);
  b.nl = big_nl(b.ntb);
  b.npad = b.ntb * kBT;
  b.rec_dir = (size_t)b.nl * kBTE;
  b.rec_neu = (size_t)b.ntb * b.ntb * kBTE;
  return b;
}

// Work arrays (doubles) of one big factorisation of nsys systems.
size_t big_factor_ws_elems(const Geometry& g, int nsys);

// Input of a big factorisation.
struct BigFactorIn {
  Geometry g;
  const double* em;      // FP64 moduli [nsys][nel]
  const uint8_t* fixed;  // supports [ndof]
  const double* K0;      // element matrix [ndpe][ndpe]
  double* dis;           // Neumann: D^-1/2 [nsub][nloc] (written); Dirichlet: unused
  double shift, fixed_diag;
  int neumann;
  int nsys;
};

// Twisted factorisation of every (system, subdomain) matrix into the
// records C_b = S_b^-1 (Schur complements of the twisted elimination).
// Dirichlet: lower tiles in C layout, element type T (double or float), out
// [nsys][nsub][nblk][rec_dir]. Neumann (nsys = 1, T = double): all tiles in A
// layout, out [nsub][nblk][rec_neu]. ws: big_factor_ws_elems(g, nsys).
template <typename T>
void big_factor(const BigFactorIn& in, T* out, double* ws, int* flag, hipStream_t st);

// zloc = A_j^-1 R_j r with the big Dirichlet records, for every running system.
template <typename T>
void big_local_solves(const Geometry& g, const double* r, const T* rec, const T* emod,
                      const uint8_t* fixed, const double* K0, T* zloc, int nsys, const Gate& gate,
                      hipStream_t st);

// Y = (shifted scaled Neumann matrix)^-1 X for every subdomain, m <= 16
// columns ([nsub][nloc][m] row-major), with the big Neumann records;
// ws: nsub * 2 * npad * 16 doubles.
void big_solve_multi(const BigFactorIn& in, const double* rec, int m, const double* X, double* Y,
                     double* ws, hipStream_t st);
inline size_t big_multi_ws_elems(const Geometry& g) {
  return (size_t)g.nsub * 2 * big_shape(g).npad * 16;
}

}  // namespace tpcg
