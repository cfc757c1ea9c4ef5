// Block-tridiagonal Cholesky factors and their triangular solves, one
// workgroup per matrix.
//
// A symmetric positive definite block-tridiagonal matrix with nblk diagonal
// blocks of size nb factors as A = L L^T with L block lower bidiagonal:
// L_bb lower triangular, B_b = L_{b,b-1}. If A has half-bandwidth w, B_{b+1}
// vanishes left of the band: B_{b+1}[r][c] = 0 for c < r - (w - nb), so it is
// an upper triangle plus pe = w - nb + 1 diagonals on and below the main one.
//
// Packed storage, one record of `bstride` elements per block row b:
//   Sq_b [nb][nb]: lower triangle (c <= r) = D_b = L_bb^-1,
//                  strict upper triangle (c > r) = B_{b+1}   (zero for the last b)
//   Bd_b [nb][pe]: Bd_b[r][t] = B_{b+1}[r][r - t]            (zero outside)
// That is exactly the band of L (plus the triangles of the inverted diagonal
// blocks, which replace the triangles of L_bb one for one). Then
//   L y = r:    y_b = D_b (r_b - B_b y_{b-1})       uses Sq_{b-1} (upper) and Sq_b (lower)
//   L^T x = y:  x_b = D_b^T (y_b - B_{b+1}^T x_{b+1})  uses Sq_b only
// and every pass reads each record once.
//
// Subdomain stiffness matrices in box order (node x fastest, then y, then z)
// are block tridiagonal with one node row (2D) or node layer (3D) per block.
#pragma once

#include "tpcg_internal.h"

namespace tpcg {

// 16-byte register vector (a native vector type, so that arrays of it stay in
// registers)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, then for the other waves. Outstanding global loads and stores
// keep flying across it (a __syncthreads would drain them as a
// workgroup-scope fence), so it may only separate threads that exchange data
// through LDS; a thread may still read back its own global writes.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

struct BtriShape {
  int nb, nblk, pe, bstride;
};

inline BtriShape btri_shape(int nb, int nblk, int w) {
  BtriShape s;
  s.nb = nb;
  s.nblk = nblk;
  s.pe = w - nb + 1 > 0 ? w - nb + 1 : 0;
  if (s.pe > nb) s.pe = nb;
  const int e = nb * nb + nb * s.pe;
  s.bstride = (e + 3) & ~3;   // 16-byte records for both FP64 and FP32
  return s;
}

// odd leading dimension: conflict-free LDS columns and rows (factorisation)
__host__ __device__ inline int lds_ld(int nb) { return nb | 1; }

template <typename T>
__host__ __device__ constexpr int stage_regs_for(int nb, int pe) {
  return ((((nb * nb + nb * pe + 3) & ~3) * (int)sizeof(T)) / 16 + kThreads - 1) / kThreads;
}

// staging register counts the kernels are instantiated for
inline int stage_bucket(int need) {
  const int b[] = {2, 5, 10, 16, 24, 36};
  for (int v : b)
    if (need <= v) return v;
  return -1;
}

__host__ __device__ inline BtriShape local_shape(const Geometry& g) {
  return {g.nb, g.nblk, g.pe, g.bstride};
}
__host__ __device__ inline BtriShape coarse_shape(const Geometry& g) {
  return {g.nbc, g.nblkc, g.pec, g.bstridec};
}

// ---------------------------------------------------------------------------
// Tiled factor storage for the single-right-hand-side subdomain solves.
//
// Since B_{b+1} = A_{b+1,b} L_bb^-T = A_{b+1,b} D_b^T, the two passes can be
// written with D_b and the stiffness coupling between node layers alone, and
// with s_b = D_b^T y_b and C_b = D_b^T D_b (the inverse of the block's Schur
// complement, symmetric) even with C_b alone:
//   L y = r:    s_b = C_b (r_b - A_{b,b-1} s_{b-1})
//   L^T x = y:  x_b = s_b - C_b (A_{b+1,b}^T x_{b+1})
// one symmetric product per block and pass. The coupling A_{b+1,b} is the
// element stiffness of the element layer between the two node layers and is
// applied matrix-free, so a record holds only the lower triangle of C_b: the
// 4 x 4 tiles (I, J), I >= J, of the block padded to 4 nt rows (diagonal
// tiles in full), tile index tau = I (I + 1) / 2 + J, element e = 4 row + col
// inside a tile. Storage is thread-major in 16-byte vectors: element e of
// tile tau sits at ((e / per) nl + tau) per + e % per, with per =
// 16 / sizeof(T), so thread tau reads its tile with 16 / per coalesced loads.
// Entries past nb are zero.
// ---------------------------------------------------------------------------
struct TileShape {
  int nb, nt, nl, tstride;   // block size, tile rows, lower tiles, elements per record
};

__host__ __device__ inline TileShape tile_shape(int nb) {
  TileShape s;
  s.nb = nb;
  s.nt = (nb + 3) / 4;
  s.nl = s.nt * (s.nt + 1) / 2;
  s.tstride = 16 * s.nl;
  return s;
}

// tau -> (I, J) with tau = I (I + 1) / 2 + J, 0 <= J <= I
__host__ __device__ inline void tile_rc(int tau, int& I, int& J) {
  int i = (int)((sqrtf(8.0f * (float)tau + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > tau) --i;
  while ((i + 1) * (i + 2) / 2 <= tau) ++i;
  I = i;
  J = tau - i * (i + 1) / 2;
}

template <typename T>
__host__ __device__ inline size_t tile_offset(int nl, int tau, int e) {
  constexpr int per = 16 / (int)sizeof(T);
  return ((size_t)(e / per) * nl + tau) * per + e % per;
}

// Input of a factorisation that computes the subdomain matrices itself from
// the element moduli (rho != nullptr): matrix j of the batch is the Dirichlet
// matrix of subdomain j (principal submatrix of the supported stiffness
// matrix on its closed-cell DOFs), or with neumann != 0 the cell-only
// stiffness matrix S = D^-1/2 K^N D^-1/2 + shift I (D = diag K^N, supported
// DOFs decoupled with diagonal fixed_diag + shift), D^-1/2 stored to dis.
// With twist set (Dirichlet matrices, tiled records only) the factorisation
// is the twisted one of the subdomain solves: the block rows above the
// middle block mid = nblk / 2 are eliminated downwards, those below it
// upwards, and block mid takes both Schur terms, so that
//   A = M M^T,  M_bb = L_bb,  M_{b,b-1} = A_{b,b-1} D_{b-1}^T (b <= mid),
//               M_{b,b+1} = A_{b,b+1} D_{b+1}^T (b >= mid);
// the records then hold C_b = D_b^T D_b of this factorisation. twist is
// scratch of nb (nb + 1) / 2 doubles per matrix.
struct StencilIn {
  Geometry g;
  const double* rho;
  const uint8_t* fixed;
  const double* K0;
  double E0, Emin, penal, shift, fixed_diag;
  int neumann;
  double* dis;
  double* twist;
  const double* emod;   // element moduli, precomputed: [nsys][nel] (launch_local_factor)
};

// factor.hip
// Packed records (tiles == false) or tiled records of C_b = D_b^T D_b only (tiles == true,
// record stride tile_shape(nb).tstride); the blocks come from A, or from the
// stencil input when si.rho is set (A is then not read).
template <typename T>
void launch_factor(const double* A, T* out, int nmat, const BtriShape& sh, int* flag,
                   hipStream_t st, bool tiles = false, const StencilIn* si = nullptr);
// Tiled records of C_b of the twisted factorisation of each subdomain's
// Dirichlet matrix, one workgroup per (subdomain, system), via the Schur
// complements (no Cholesky factor): moduli of system s at si.emod + s nel,
// its records at out + s ostride, scratch si.twist [nsys][nsub][nb (nb+1)/2]
// (optional). local_factor_fits tells whether it takes geometry g (block
// size and LDS).
bool local_factor_fits(const Geometry& g);
template <typename T>
void launch_local_factor(const StencilIn& si, T* out, int* flag, int nsys, size_t ostride,
                         hipStream_t st);
void launch_solve_multi(const double* fac, const BtriShape& sh, int nmat, int m, const double* X,
                        double* Y, hipStream_t st);
// dense symmetric inverse [nmat][n][n] of packed factors (n = nb * nblk)
void launch_inverse(const double* fac, const BtriShape& sh, int nmat, double* Xinv,
                    hipStream_t st);

// (A_{b+1,b} v)[o] for a DOF o of node layer b + 1 (top = true, v on layer b)
// or (A_{b+1,b}^T v)[o] = (A_{b,b+1} v)[o] for a DOF o of layer b (top =
// false, v on layer b + 1): the stiffness of the element layer between the
// two node layers, E[] its moduli indexed (ex + 1) + (bn + 1) (ey + 1) over
// box-local element coordinates, zero outside the mesh. Supported DOFs are
// masked by the caller.
template <typename T>
__device__ inline T layer_coupling(int d, int bn, const T* __restrict__ K0s,
                                   const T* __restrict__ E, const T* __restrict__ v, int o,
                                   bool top) {
  const int nd = d == 3 ? 24 : 8;
  const int m = o / d, c = o - m * d;
  const int lx = m % bn, ly = d == 3 ? m / bn : 0;
  const int ny = d == 3 ? 2 : 1, ylim = d == 3 ? bn : 1;
  T acc = 0;
  for (int hy = 0; hy < ny; ++hy)
    for (int hx = 0; hx < 2; ++hx) {
      // element with this node at its corner (hx, hy) of the top or bottom face
      const int ex = lx - hx, ey = ly - hy;
      const T Ee = E[(ex + 1) + (d == 3 ? (bn + 1) * (ey + 1) : 0)];
      const int ca = d == 3 ? corner_of(hx, hy, top) : corner_of(hx, top, 0);
      T s = 0;
      for (int oy = 0; oy < ny; ++oy)
        for (int ox = 0; ox < 2; ++ox) {
          const int px = ex + ox, py = ey + oy;
          if (px < 0 || px >= bn || py < 0 || py >= ylim) continue;
          const int cb = d == 3 ? corner_of(ox, oy, !top) : corner_of(ox, !top, 0);
          const T* kr = K0s + (d * ca + c) * nd + d * cb;
          const T* vp = v + d * (px + bn * py);
          for (int c2 = 0; c2 < d; ++c2) s += kr[c2] * vp[c2];
        }
      acc += Ee * s;
    }
  return acc;
}

// layer_coupling with the dimension fixed at compile time and the DOF's
// position in the layer (node lx, ly, component c) decoded once by the
// caller: the loops unroll, so the LDS reads of a call are issued together
// instead of one after another. Same terms, same order of summation.
template <int D, typename T>
__device__ inline T layer_coupling_at(int bn, const T* __restrict__ K0s, const T* __restrict__ E,
                                      const T* __restrict__ v, int lx, int ly, int c, bool top) {
  constexpr int nd = D == 3 ? 24 : 8, ny = D == 3 ? 2 : 1;
  const int ylim = D == 3 ? bn : 1;
  T acc = 0;
#pragma unroll
  for (int hy = 0; hy < ny; ++hy)
#pragma unroll
    for (int hx = 0; hx < 2; ++hx) {
      const int ex = lx - hx, ey = ly - hy;
      const T Ee = E[(ex + 1) + (D == 3 ? (bn + 1) * (ey + 1) : 0)];
      const int ca = D == 3 ? corner_of(hx, hy, top) : corner_of(hx, top, 0);
      T s = 0;
#pragma unroll
      for (int oy = 0; oy < ny; ++oy)
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
          const int px = ex + ox, py = ey + oy;
          if (px < 0 || px >= bn || py < 0 || py >= ylim) continue;
          const int cb = D == 3 ? corner_of(ox, oy, !top) : corner_of(ox, !top, 0);
          const T* kr = K0s + (D * ca + c) * nd + D * cb;
          const T* vp = v + D * (px + bn * py);
#pragma unroll
          for (int c2 = 0; c2 < D; ++c2) s += kr[c2] * vp[c2];
        }
      acc += Ee * s;
    }
  return acc;
}

// LDS element count of btri_solve for shape s and NR right-hand sides
__host__ __device__ inline size_t btri_solve_lds_elems(const BtriShape& s, int nr) {
  return (size_t)s.bstride + 2 * (size_t)s.nb * nr + (size_t)kThreads * nr;
}

// Partial sums of one of the four triangular products for all nr columns of
// v ([nb][nr] row-major) into red[q][i][r]: thread t owns output row (or
// column) i = t % nb over the chunk q = t / nb of the summation index.
//   MODE 0: y = lower(M) v            MODE 2: y = lower(M)^T v
//   MODE 1: y = (upper(M) + band) v   MODE 3: y = (upper(M) + band)^T v
// upper(M) is the strict upper triangle; band[i][t] multiplies v[i - t].
template <typename T, int NR, int MODE>
__device__ inline void tri_parts(const T* __restrict__ M, int ld, const T* __restrict__ E, int pe,
                                 int nb, const T* __restrict__ v, int nr, T* __restrict__ red) {
  const int t = threadIdx.x;
  const int Q = kThreads / nb;
  const int L = (nb + Q - 1) / Q;
  const int i = t % nb, q = t / nb;
  if (q >= Q) return;
  T acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0;
  const int c0 = q * L, c1 = min(nb, c0 + L);
  int lo, hi;
  if (MODE == 0) { lo = c0; hi = min(c1, i + 1); }
  else if (MODE == 1) { lo = max(c0, i + 1); hi = c1; }
  else if (MODE == 2) { lo = max(c0, i); hi = c1; }
  else { lo = c0; hi = min(c1, i); }
  for (int c = lo; c < hi; ++c) {
    const T a = (MODE < 2) ? M[i * ld + c] : M[c * ld + i];
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nr) acc[r] += a * v[c * nr + r];
  }
  if (q == 0) {
    if (MODE == 1) {
      for (int tt = 0; tt < pe && i - tt >= 0; ++tt) {
        const T a = E[i * pe + tt];
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr) acc[r] += a * v[(i - tt) * nr + r];
      }
    } else if (MODE == 3) {
      for (int tt = 0; tt < pe && i + tt < nb; ++tt) {
        const T a = E[(i + tt) * pe + tt];
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr) acc[r] += a * v[(i + tt) * nr + r];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r < nr) red[((size_t)q * nb + i) * nr + r] = acc[r];
}

template <typename T>
__device__ inline T red_sum(const T* red, int nb, int nr, int i, int r) {
  const int Q = kThreads / nb;
  T s = 0;
  for (int q = 0; q < Q; ++q) s += red[((size_t)q * nb + i) * nr + r];
  return s;
}

// Solve (L L^T) X = R for one packed factor `fac` ([nblk][bstride] of T) and
// nr <= NR right-hand sides. rhs(b, i, r) returns R's element (row i of block
// b, column r); out(b, i, r) is a T slot receiving Y (forward) and then X.
// Each vector element is handled by one fixed thread in both passes, so the
// reads of Y in the backward pass see that thread's own forward writes.
template <typename T, int NR, int MAXV, typename Rhs, typename Out>
__device__ void btri_solve(const T* __restrict__ fac, const BtriShape sh, int nr, Rhs rhs, Out out,
                           unsigned char* smem) {
  const int nb = sh.nb, nblk = sh.nblk, pe = sh.pe;
  const int ld = nb;                              // LDS holds the record as stored
  T* M = reinterpret_cast<T*>(smem);
  T* E = M + (size_t)nb * nb;
  T* va = M + sh.bstride;
  T* vb = va + (size_t)nb * nr;
  T* red = vb + (size_t)nb * nr;
  const int nv = sh.bstride * (int)sizeof(T) / 16;
  const int t = threadIdx.x;
  const int nvec = nb * nr;                       // vector elements per block
  constexpr int VR = (kMaxNb * NR + kThreads - 1) / kThreads;
  u32x4 stg[MAXV];                                // register staging of the next record
  T vreg[VR];
  auto rec = [&](int b) { return fac + (size_t)b * sh.bstride; };
#define TPCG_STAGE_LOAD(b_)                                                   \
  {                                                                           \
    const u32x4* s_ = reinterpret_cast<const u32x4*>(rec(b_));                \
    _Pragma("unroll") for (int k_ = 0; k_ < MAXV; ++k_) {                     \
      const int idx_ = t + k_ * kThreads;                                     \
      if (idx_ < nv) stg[k_] = s_[idx_];                                      \
    }                                                                         \
  }
#define TPCG_STAGE_STORE()                                                    \
  {                                                                           \
    u32x4* d_ = reinterpret_cast<u32x4*>(M);                                  \
    _Pragma("unroll") for (int k_ = 0; k_ < MAXV; ++k_) {                     \
      const int idx_ = t + k_ * kThreads;                                     \
      if (idx_ < nv) d_[idx_] = stg[k_];                                      \
    }                                                                         \
  }
  auto vload_rhs = [&](int b) {
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int e = t + u * kThreads;
      if (e < nvec) vreg[u] = (T)rhs(b, e / nr, e % nr);
    }
  };
  auto vload_out = [&](int b) {
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int e = t + u * kThreads;
      if (e < nvec) vreg[u] = out(b, e / nr, e % nr);
    }
  };
  auto vstore = [&](T* dst) {
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int e = t + u * kThreads;
      if (e < nvec) dst[e] = vreg[u];
    }
  };
  // combine the chunk partials into dst (minus: dst = base - sum), and
  // optionally write the result to `out` for block b
  auto combine = [&](T* dst, const T* base, bool minus, int b, bool write) {
    for (int e = t; e < nvec; e += kThreads) {
      const int i = e / nr, r = e - (e / nr) * nr;
      const T s = red_sum(red, nb, nr, i, r);
      const T v = minus ? base[e] - s : s;
      dst[e] = v;
      if (write) out(b, i, r) = v;
    }
  };

  // ---- forward: y_b = D_b (r_b - B_b y_{b-1}) ----
  TPCG_STAGE_LOAD(0);
  vload_rhs(0);
  TPCG_STAGE_STORE();
  vstore(va);
  if (nblk > 1) { TPCG_STAGE_LOAD(1); vload_rhs(1); }
  __syncthreads();
  tri_parts<T, NR, 0>(M, ld, E, pe, nb, va, nr, red);
  __syncthreads();
  combine(vb, nullptr, false, 0, true);
  for (int b = 1; b < nblk; ++b) {
    __syncthreads();
    vstore(va);                                        // r_b
    __syncthreads();
    tri_parts<T, NR, 1>(M, ld, E, pe, nb, vb, nr, red);   // B_b from record b-1
    __syncthreads();
    combine(va, va, true, b, false);
    __syncthreads();
    TPCG_STAGE_STORE();           // record b
    if (b + 1 < nblk) { TPCG_STAGE_LOAD(b + 1); vload_rhs(b + 1); }
    else if (nblk > 1) { TPCG_STAGE_LOAD(nblk - 2); }
    __syncthreads();
    tri_parts<T, NR, 0>(M, ld, E, pe, nb, va, nr, red);
    __syncthreads();
    combine(vb, nullptr, false, b, true);
  }
  // ---- backward: x_b = D_b^T (y_b - B_{b+1}^T x_{b+1}) ----
  __syncthreads();
  tri_parts<T, NR, 2>(M, ld, E, pe, nb, vb, nr, red);
  __syncthreads();
  combine(vb, nullptr, false, nblk - 1, true);
  if (nblk > 1) vload_out(nblk - 2);
  for (int b = nblk - 2; b >= 0; --b) {
    __syncthreads();
    TPCG_STAGE_STORE();           // record b
    vstore(va);                                        // y_b
    if (b >= 1) { TPCG_STAGE_LOAD(b - 1); vload_out(b - 1); }
    __syncthreads();
    tri_parts<T, NR, 3>(M, ld, E, pe, nb, vb, nr, red);   // B_{b+1}^T from record b
    __syncthreads();
    combine(va, va, true, b, false);
    __syncthreads();
    tri_parts<T, NR, 2>(M, ld, E, pe, nb, va, nr, red);
    __syncthreads();
    combine(vb, nullptr, false, b, true);
  }
  __syncthreads();
#undef TPCG_STAGE_LOAD
#undef TPCG_STAGE_STORE
}

// ---------------------------------------------------------------------------
// The same solve for up to 16 right-hand sides in FP64 on the matrix cores:
// every product of a record with a block of the right-hand sides is a set of
// 16 x 16 output tiles (v_mfma_f64_16x16x4f64; A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k, D[i][j] in lane j + 16 (i % 4), register i / 4),
// one row tile per wave. The triangular masks and the band are applied when
// the A operand is fetched.
// ---------------------------------------------------------------------------
typedef double dvec4 __attribute__((ext_vector_type(4)));

// Address of element (r, c) of the operand, clamped into the record, and
// whether the element is inside the matrix, the triangle or the band (else
// it is zero).
template <int MODE>
__device__ inline const double* rec_addr(const double* M, const double* E, int nb, int pe, int r,
                                         int c, bool& ok) {
  const int rr = min(r, nb - 1), cc = min(c, nb - 1);
  const bool in = r < nb && c < nb;
  if (MODE == 0) { ok = in && c <= r; return M + rr * nb + cc; }
  if (MODE == 2) { ok = in && r <= c; return M + cc * nb + rr; }
  // B_b from the strict upper triangle of M and the band E
  const int lo = MODE == 1 ? rr : cc, hi = MODE == 1 ? cc : rr;   // row / column of M
  const int off = lo - hi;                                          // > 0 below the diagonal
  const bool up = hi > lo;
  ok = in && (up || off < pe);
  return up ? M + lo * nb + hi : E + lo * pe + min(max(off, 0), pe - 1);
}

// dst = op(M) v  (or base - op(M) v); v, dst, base are [npad][16] in LDS.
// The wave index is made uniform so that the tile and k loops are scalar
// loops and the accumulator stays in place between MFMAs. The operands of
// four k-steps are read unconditionally from clamped addresses (the empty asm
// keeps the compiler from moving the reads under their masks, which would
// serialise them) and masked after one wait.
template <int MODE>
__device__ inline void rec_gemm16(const double* M, const double* E, int nb, int pe, int npad,
                                  const double* v, double* dst, const double* base) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  const int li = l & 15, lq = l >> 4;
  for (int I = wv; 16 * I < npad; I += 4) {
    int k0 = 0, k1 = npad;
    if (MODE == 0) k1 = min(npad, 16 * I + 16);
    if (MODE == 1) k0 = max(0, (16 * I - pe + 1) & ~3);
    if (MODE == 2) k0 = 16 * I;
    if (MODE == 3) k1 = min(npad, (16 * I + 15 + pe + 3) & ~3);
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
    const int r = 16 * I + li;
    int k = k0;
    for (; k + 16 <= k1; k += 16) {
      double a[4], b[4];
      bool ok[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = *rec_addr<MODE>(M, E, nb, pe, r, k + 4 * u + lq, ok[u]);
        b[u] = v[(k + 4 * u + lq) * 16 + li];
      }
      asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]));
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ok[u] ? a[u] : 0.0, b[u], acc, 0, 0, 0);
    }
    for (; k < k1; k += 4) {
      bool ok;
      double a = *rec_addr<MODE>(M, E, nb, pe, r, k + lq, ok);
      const double b = v[(k + lq) * 16 + li];
      asm volatile("" : "+v"(a));
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ok ? a : 0.0, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rq = 16 * I + 4 * q + lq;
      dst[rq * 16 + li] = base ? base[rq * 16 + li] - acc[q] : acc[q];
    }
  }
}

__host__ __device__ inline size_t btri_solve16_lds_elems(const BtriShape& s) {
  const int npad = (s.nb + 15) & ~15;
  return (size_t)s.bstride + 2 * (size_t)npad * 16;
}

// b0: the right-hand sides vanish in the blocks before b0 (so does y there):
// the forward sweep starts at b0 and the backward sweep takes y_b = 0 below
// it without reading out.
template <int MAXV, typename Rhs, typename Out>
__device__ void btri_solve16(const double* __restrict__ fac, const BtriShape sh, int nr, Rhs rhs,
                             Out out, unsigned char* smem, int b0 = 0) {
  const int nb = sh.nb, nblk = sh.nblk, pe = sh.pe;
  const int npad = (nb + 15) & ~15;
  double* M = reinterpret_cast<double*>(smem);
  double* E = M + (size_t)nb * nb;
  double* va = M + sh.bstride;
  double* vb = va + (size_t)npad * 16;
  const int nv = sh.bstride * (int)sizeof(double) / 16;
  const int t = threadIdx.x;
  const int nvec = npad * 16;
  constexpr int VR = ((kMaxNb + 15) / 16 * 16 * 16 + kThreads - 1) / kThreads;
  u32x4 stg[MAXV];
  double vreg[VR];
  auto rec = [&](int b) { return fac + (size_t)b * sh.bstride; };
  auto stage_load = [&](int b) {
    const u32x4* s = reinterpret_cast<const u32x4*>(rec(b));
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const int idx = t + k * kThreads;
      if (idx < nv) stg[k] = s[idx];
    }
  };
  auto stage_store = [&]() {
    u32x4* d = reinterpret_cast<u32x4*>(M);
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const int idx = t + k * kThreads;
      if (idx < nv) d[idx] = stg[k];
    }
  };
  auto vload_rhs = [&](int b) {
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int e = t + u * kThreads;
      const int i = e >> 4, r = e & 15;
      if (e < nvec) vreg[u] = (i < nb && r < nr) ? rhs(b, i, r) : 0.0;
    }
  };
  auto vload_out = [&](int b) {
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int e = t + u * kThreads;
      const int i = e >> 4, r = e & 15;
      if (e < nvec) vreg[u] = (b >= b0 && i < nb && r < nr) ? out(b, i, r) : 0.0;
    }
  };
  auto vstore = [&](double* dst) {
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int e = t + u * kThreads;
      if (e < nvec) dst[e] = vreg[u];
    }
  };
  auto write_out = [&](const double* src, int b) {
    for (int e = t; e < nvec; e += kThreads) {
      const int i = e >> 4, r = e & 15;
      if (i < nb && r < nr) out(b, i, r) = src[e];
    }
  };
  // forward, from block b0 (y_{b0-1} = 0)
  stage_load(b0);
  vload_rhs(b0);
  stage_store();
  vstore(va);
  if (b0 + 1 < nblk) { stage_load(b0 + 1); vload_rhs(b0 + 1); }
  else if (nblk > 1) { stage_load(nblk - 2); }
  __syncthreads();
  rec_gemm16<0>(M, E, nb, pe, npad, va, vb, nullptr);
  __syncthreads();
  write_out(vb, b0);
  for (int b = b0 + 1; b < nblk; ++b) {
    vstore(va);                                   // r_b (va last read before the barrier)
    __syncthreads();
    rec_gemm16<1>(M, E, nb, pe, npad, vb, va, va);   // t_b = r_b - B_b y_{b-1}
    __syncthreads();
    stage_store();                                // record b
    if (b + 1 < nblk) { stage_load(b + 1); vload_rhs(b + 1); }
    else if (nblk > 1) { stage_load(nblk - 2); }
    __syncthreads();
    rec_gemm16<0>(M, E, nb, pe, npad, va, vb, nullptr);
    __syncthreads();
    write_out(vb, b);
  }
  // backward
  rec_gemm16<2>(M, E, nb, pe, npad, vb, va, nullptr);   // x_{n-1}
  __syncthreads();
  write_out(va, nblk - 1);
  {
    // move x_{n-1} into vb
    for (int e = t; e < nvec; e += kThreads) vb[e] = va[e];
  }
  if (nblk > 1) vload_out(nblk - 2);
  for (int b = nblk - 2; b >= 0; --b) {
    __syncthreads();
    stage_store();                                // record b
    vstore(va);                                   // y_b
    if (b >= 1) { stage_load(b - 1); vload_out(b - 1); }
    __syncthreads();
    rec_gemm16<3>(M, E, nb, pe, npad, vb, va, va);   // s_b = y_b - B_{b+1}^T x_{b+1}
    __syncthreads();
    rec_gemm16<2>(M, E, nb, pe, npad, va, vb, nullptr);   // x_b = D_b^T s_b
    __syncthreads();
    write_out(vb, b);
  }
  __syncthreads();
}

}  // namespace tpcg
