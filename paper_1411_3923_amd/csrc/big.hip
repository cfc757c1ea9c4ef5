// HBM-resident batched kernels for subdomain blocks beyond the on-chip factor
// kernels (3-d cells of 16^3 elements: node-layer blocks of 867 unknowns) and
// for the dense coarse matrix (Sec. 2.4 coarse projection equation).
//
// Local factors (Sec. 2.4.2, two-level additive Schwarz: exact solves with
// the principal submatrices A_j; Sec. 2.4 and Sec. 3.2 for the scaled
// Neumann matrices of the eigenproblems). The box matrix is block
// tridiagonal over its node layers and is eliminated in twisted order (the
// layers above the middle block downwards, those below it upwards, the
// middle block taking both Schur terms); a record holds
//   C_b = S_b^-1,  S_b = A_bb - A_{b,p} C_p A_{p,b}  (p: the previous block of b's half).
// Per level of the elimination (one block of each half for every system
// and subdomain):
//   1. T = (A_{b,p} C_p)^T, a 27-point layer-coupling stencil applied to the
//      rows of C_p (a window of three node rows in LDS);
//   2. S_b = A_bb - A_{b,p} T, the same stencil on the rows of T, A_bb formed
//      on the fly from the element moduli;
//   3. S_b^-1 by the symmetric block sweep (below) on the matrix cores;
//   4. the records, in the solve's layout and precision.
//
// Symmetric block sweep: for pivot tiles K = 0 .. ntb - 1, with P = A_KK,
//   A_ij -= A_iK P^-1 A_Kj (i, j not in K),  A_iK <- A_iK P^-1,
//   A_Kj <- P^-1 A_Kj,                       A_KK <- -P^-1,
// which leaves -A^-1 after the last pivot. Only the lower tiles are kept; a
// step is three launches: P^-1 by Gauss-Jordan elimination in LDS (one
// workgroup per matrix), the panels V_I = A_IK and W_I = V_I P^-1 (one
// workgroup per tile row), and the rank-64 update S_IJ -= W_I V_J^T of
// every lower tile (one workgroup per tile, v_mfma_f64_16x16x4f64 with both
// operands read as coalesced 512-byte fragments).
#include <algorithm>
#include <utility>

#include "big.h"
#include "btri.h"

namespace tpcg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// (r, c) of the element at C-layout offset o
__device__ inline void cdec(int o, int& r, int& c) {
  const int lane = o & 63, reg = o >> 6;
  r = 16 * (reg >> 4) + 4 * (reg & 3) + (lane >> 4);
  c = 16 * ((reg >> 2) & 3) + (lane & 15);
}
// (r, c) of the element at A-layout offset o
__device__ inline void adec(int o, int& r, int& c) {
  const int lane = o & 63, frag = o >> 6;
  r = 16 * (frag >> 4) + (lane & 15);
  c = 4 * (frag & 15) + (lane >> 4);
}

// ---------------------------------------------------------------------------
// Symmetric block sweep
// ---------------------------------------------------------------------------

// P^-1 of the pivot tile of every matrix by the symmetric sweep of its 64
// pivots, one wave per matrix: lane j keeps column j in registers; at step k
// every lane publishes its entry of row k (= column k, the sweep keeps the
// matrix symmetric), then
//   a_ij -= a_ik a_kj / p,  a_ik <- a_ik / p,  a_kj <- a_kj / p,  a_kk <- -1/p
// (p = a_kk > 0 for an SPD tile, the Schur complements' diagonals). After
// the 64th step the tile holds -P^-1; P^-1 is written row-major.
__global__ __launch_bounds__(64) void k_sw_pivot(const double* __restrict__ S, size_t mstride,
                                                 int K, double* __restrict__ pinv,
                                                 int* __restrict__ flag) {
  __shared__ double col[kBT];
  const int m = blockIdx.x, j = threadIdx.x;
  const double* src = S + (size_t)m * mstride + (size_t)big_ltile(K, K) * kBTE;
  // a[i] holds row (i + 8 kb) mod 64 of column j: the array turns by 8 after
  // every block of 8 pivots, so that pivot row 8 kb + kk sits at a[kk] and
  // every register index is a constant
  double a[kBT];
#pragma unroll
  for (int i = 0; i < kBT; ++i) a[i] = src[big_cofs(i, j)];
  bool bad = false;
  for (int kb = 0; kb < kBT / 8; ++kb) {
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 8 * kb + kk;
      const double akj = a[kk];
      col[j] = akj;
      __syncthreads();
      double p = col[k];
      if (!(p > 0.0)) {
        bad = true;
        p = 1.0;
      }
      const double ip = 1.0 / p;
      const double sk = akj * ip;       // a_kj / p
#pragma unroll
      for (int i = 0; i < kBT; ++i) {
        if (i == kk) continue;
        const double aik = col[(i + 8 * kb) & (kBT - 1)];
        a[i] = j == k ? aik * ip : a[i] - aik * sk;
      }
      a[kk] = j == k ? -ip : sk;
      __syncthreads();
    }
    double t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = a[i];
#pragma unroll
    for (int i = 0; i < kBT - 8; ++i) a[i] = a[i + 8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[kBT - 8 + i] = t[i];
  }
  if (bad && j == 0) flag[0] = 1;
  double* dst = pinv + (size_t)m * kBTE;
#pragma unroll
  for (int i = 0; i < kBT; ++i) dst[i * kBT + j] = -a[i];
}

// Panels of step K for tile row I != K: V_I = A_IK (from tile (I, K), or
// the transpose of tile (K, I) above the diagonal) and W_I = V_I P^-1 on the
// matrix cores, both written in A layout. grid (ntb, nmat).
__global__ __launch_bounds__(kThreads) void k_sw_panel(const double* __restrict__ S,
                                                      size_t mstride, int ntb, int K,
                                                      const double* __restrict__ pinv,
                                                      double* __restrict__ Wp,
                                                      double* __restrict__ Vp) {
  __shared__ double Vl[kBT][kBT + 1];
  __shared__ double Pl[kBT][kBT + 1];
  const int I = blockIdx.x, m = blockIdx.y, t = threadIdx.x;
  if (I == K) return;
  const double* Sm = S + (size_t)m * mstride;
  const bool below = I > K;
  const double* src = Sm + (size_t)(below ? big_ltile(I, K) : big_ltile(K, I)) * kBTE;
  const double* pv = pinv + (size_t)m * kBTE;
  for (int o = t; o < kBTE; o += kThreads) {
    int r, c;
    cdec(o, r, c);
    const double v = src[o];
    if (below) Vl[r][c] = v;
    else Vl[c][r] = v;
    Pl[o >> 6][o & 63] = pv[o];
  }
  __syncthreads();
  const int w = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63, li = l & 15, lk = l >> 4;
  d4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int ks = 0; ks < 16; ++ks) {
    const double a = Vl[16 * w + li][4 * ks + lk];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma4(a, Pl[4 * ks + lk][16 * cb + li], acc[cb]);
  }
  __syncthreads();
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) Pl[16 * w + 4 * v + lk][16 * cb + li] = acc[cb][v];
  __syncthreads();
  double* Wd = Wp + ((size_t)m * ntb + I) * kBTE;
  double* Vd = Vp + ((size_t)m * ntb + I) * kBTE;
  for (int o = t; o < kBTE; o += kThreads) {
    int r, c;
    adec(o, r, c);
    Wd[o] = Pl[r][c];
    Vd[o] = Vl[r][c];
  }
}

// Update of step K, one workgroup per lower tile (I, J): S_IJ -= W_I V_J^T
// off row and column K (wave w: rows 16 w .. + 15, accumulators loaded from
// and stored to the tile); tile (I, K) <- W_I, tile (K, J) <- W_J^T,
// tile (K, K) <- -P^-1. grid (nl, nmat).
__global__ __launch_bounds__(kThreads) void k_sw_update(double* __restrict__ S, size_t mstride,
                                                       int ntb, int K,
                                                       const double* __restrict__ pinv,
                                                       const double* __restrict__ Wp,
                                                       const double* __restrict__ Vp) {
  const int q = blockIdx.x, m = blockIdx.y, t = threadIdx.x;
  int I, J;
  tile_rc(q, I, J);
  double* T = S + (size_t)m * mstride + (size_t)q * kBTE;
  const double* Wm = Wp + (size_t)m * ntb * kBTE;
  const double* Vm = Vp + (size_t)m * ntb * kBTE;
  if (I != K && J != K) {
    const int w = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63;
    double* Tw = T + (size_t)w * 16 * 64;
    d4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[cb][v] = Tw[(cb * 4 + v) * 64 + l];
    const double* WI = Wm + (size_t)I * kBTE + (size_t)w * 16 * 64;
    const double* VJ = Vm + (size_t)J * kBTE;
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
      double a[4], b[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = WI[(k0 + u) * 64 + l];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) b[u][cb] = VJ[(cb * 16 + k0 + u) * 64 + l];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma4(-a[u], b[u][cb], acc[cb]);
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) Tw[(cb * 4 + v) * 64 + l] = acc[cb][v];
    return;
  }
  for (int o = t; o < kBTE; o += kThreads) {
    int r, c;
    cdec(o, r, c);
    double v;
    if (I == K && J == K) v = -pinv[(size_t)m * kBTE + r * kBT + c];
    else if (J == K) v = Wm[(size_t)I * kBTE + big_aofs(r, c)];
    else v = Wm[(size_t)J * kBTE + big_aofs(c, r)];
    T[o] = v;
  }
}

// ---------------------------------------------------------------------------
// Dense coarse matrix
// ---------------------------------------------------------------------------

// Lower tiles of K_c (C layout) from the block-tridiagonal assembly
// (diagonal blocks in full, sub-diagonal blocks A_{b,b-1}); identity past nt.
__global__ __launch_bounds__(kThreads) void k_coarse_expand(Geometry g, const double* __restrict__ Ac,
                                                           size_t astride, double* __restrict__ S,
                                                           size_t mstride) {
  const int q = blockIdx.x, sys = blockIdx.y;
  int I, J;
  tile_rc(q, I, J);
  const double* A = Ac + (size_t)sys * astride;
  double* T = S + (size_t)sys * mstride + (size_t)q * kBTE;
  const int nt = g.nt, nbc = g.nbc;
  const size_t bsz = (size_t)nbc * nbc;
  for (int o = threadIdx.x; o < kBTE; o += kThreads) {
    int r, c;
    cdec(o, r, c);
    const int R = kBT * I + r, C = kBT * J + c;
    double v;
    if (R >= nt || C >= nt) {
      v = R == C ? 1.0 : 0.0;
    } else {
      const int rb = R / nbc, cb = C / nbc, ri = R - rb * nbc, ci = C - cb * nbc;
      if (rb == cb) v = A[(size_t)(2 * rb) * bsz + (size_t)ri * nbc + ci];
      else if (rb == cb + 1) v = A[(size_t)(2 * rb + 1) * bsz + (size_t)ri * nbc + ci];
      else if (cb == rb + 1) v = A[(size_t)(2 * cb + 1) * bsz + (size_t)ci * nbc + ri];
      else v = 0.0;
    }
    T[o] = v;
  }
}

// Lower tiles of K_c^-1 (row-major in each tile, zero past nt) from the
// sweep's -K_c^-1.
__global__ __launch_bounds__(kThreads) void k_coarse_store(Geometry g, const double* __restrict__ S,
                                                          size_t mstride, int nl,
                                                          double* __restrict__ cpk) {
  const int q = blockIdx.x, sys = blockIdx.y;
  int I, J;
  tile_rc(q, I, J);
  const double* T = S + (size_t)sys * mstride + (size_t)q * kBTE;
  double* D = cpk + ((size_t)sys * nl + q) * kBTE;
  const int nt = g.nt;
  for (int e = threadIdx.x; e < kBTE; e += kThreads) {
    const int r = e >> 6, c = e & 63;
    const int R = kBT * I + r, C = kBT * J + c;
    D[e] = (R < nt && C < nt) ? -T[big_cofs(r, c)] : 0.0;
  }
}

// Lower tiles of K_c^-1 (row-major in each tile, zero past nt) from a dense
// row-major K_c^-1 [nsys][nt][nt] (the block-tridiagonal path's inverse).
__global__ __launch_bounds__(kThreads) void k_coarse_pack(Geometry g, const double* __restrict__ inv,
                                                         int nl, double* __restrict__ cpk) {
  const int q = blockIdx.x, sys = blockIdx.y, nt = g.nt;
  int I, J;
  tile_rc(q, I, J);
  const double* src = inv + (size_t)sys * nt * nt;
  double* dst = cpk + ((size_t)sys * nl + q) * kBTE;
  for (int e = threadIdx.x; e < kBTE; e += kThreads) {
    const int r = kBT * I + (e >> 6), c = kBT * J + (e & 63);
    dst[e] = (r < nt && c < nt) ? src[(size_t)r * nt + c] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Coarse matrix as an HBM-resident block-tridiagonal factorisation (coarse
// spaces too large for a dense inverse, with blocks too large for the on-chip
// kernels). K_c = L D L^T with D = diag(S_b), L_{b+1,b} = A_{b+1,b} S_b^-1.
// A window of two block rows holds [S_b; A_{b+1,b} A_{b+1,b+1}] as lower
// tiles; sweeping only the first block's pivots leaves -S_b^-1 in the first
// block, L_{b+1,b} below it and S_{b+1} in the second, which then moves up.
// Stored per system, row-major nbc x nbc: S_b^-1, L_{b,b-1} and L_{b+1,b}^T.
// ---------------------------------------------------------------------------

// tiles of block row b + 1 of the window (second = 1: the coupling and
// diagonal blocks of block row b + 1 of the assembly; second = 0, first
// block: A_00), identity on the padding. grid (nl2, nsys).
__global__ __launch_bounds__(kThreads) void k_cb_fill(Geometry g, const double* __restrict__ Ac,
                                                     size_t astride, int br, int ntb, int second,
                                                     double* __restrict__ W, size_t wstride) {
  const int q = blockIdx.x, sys = blockIdx.y;
  int I, J;
  tile_rc(q, I, J);
  const bool lead = I < ntb;                      // tile of the first block
  if (second ? lead : !lead) return;
  const double* A = Ac + (size_t)sys * astride;
  const int nbc = g.nbc;
  const size_t bsz = (size_t)nbc * nbc;
  double* T = W + (size_t)sys * wstride + (size_t)q * kBTE;
  for (int o = threadIdx.x; o < kBTE; o += kThreads) {
    int r, c;
    cdec(o, r, c);
    const int R = kBT * (lead ? I : I - ntb) + r;     // row in its block
    const bool cdiag = !lead && J >= ntb;
    const int C = kBT * (cdiag ? J - ntb : J) + c;
    double v;
    if (lead) {
      v = (R < nbc && C < nbc) ? A[(size_t)(2 * br) * bsz + (size_t)R * nbc + C] : (R == C ? 1.0 : 0.0);
    } else if (cdiag) {
      v = (R < nbc && C < nbc) ? A[(size_t)(2 * br) * bsz + (size_t)R * nbc + C] : (R == C ? 1.0 : 0.0);
    } else {
      v = (R < nbc && C < nbc) ? A[(size_t)(2 * br + 1) * bsz + (size_t)R * nbc + C] : 0.0;
    }
    T[o] = v;
  }
}

// second block -> first block (tile (I, J), I, J >= ntb, to (I - ntb, J -
// ntb); the targets lie before every source in tile order). grid (nl, nsys).
__global__ __launch_bounds__(kThreads) void k_cb_shift(int ntb, double* __restrict__ W,
                                                      size_t wstride) {
  const int q = blockIdx.x, sys = blockIdx.y;
  int I, J;
  tile_rc(q, I, J);   // tile of the first block
  double* Wm = W + (size_t)sys * wstride;
  const double* src = Wm + (size_t)big_ltile(I + ntb, J + ntb) * kBTE;
  double* dst = Wm + (size_t)q * kBTE;
  for (int o = threadIdx.x; o < kBTE; o += kThreads) dst[o] = src[o];
}

// S_b^-1 = -(first block) and, with coupling = 1, L_{b+1,b} (the tiles below
// it) and its transpose, row-major and trimmed to nbc. grid (nl2, nsys).
__global__ __launch_bounds__(kThreads) void k_cb_extract(Geometry g, const double* __restrict__ W,
                                                        size_t wstride, int ntb, int b,
                                                        int coupling, double* __restrict__ cband) {
  const int q = blockIdx.x, sys = blockIdx.y;
  int I, J;
  tile_rc(q, I, J);
  const int nbc = g.nbc, nblk = g.nblkc;
  const size_t bsz = (size_t)nbc * nbc;
  double* base = cband + (size_t)sys * 3 * nblk * bsz;
  double* Si = base + (size_t)b * bsz;
  double* Lf = base + (size_t)(nblk + b + 1) * bsz;    // L_{b+1,b}
  double* Lt = base + (size_t)(2 * nblk + b) * bsz;    // L_{b+1,b}^T
  const double* T = W + (size_t)sys * wstride + (size_t)q * kBTE;
  const bool lead = I < ntb;
  if (!lead && (!coupling || J >= ntb)) return;
  for (int o = threadIdx.x; o < kBTE; o += kThreads) {
    int r, c;
    cdec(o, r, c);
    const double v = T[o];
    if (lead) {
      // one triangle of a diagonal tile gives both halves (its two halves
      // agree only up to rounding)
      if (I == J && r < c) continue;
      const int R = kBT * I + r, C = kBT * J + c;
      if (R < nbc && C < nbc) {
        Si[(size_t)R * nbc + C] = -v;
        Si[(size_t)C * nbc + R] = -v;
      }
    } else {
      const int R = kBT * (I - ntb) + r, C = kBT * J + c;
      if (R < nbc && C < nbc) {
        Lf[(size_t)R * nbc + C] = v;
        Lt[(size_t)C * nbc + R] = v;
      }
    }
  }
}

// out = a - M v (a null: out = M v) for the nbc x nbc row-major blocks M of
// every running system: block blockIdx.y of a batch, at stride bstride in M,
// a, v and out (bvstride); eight rows per workgroup, two per wave.
// grid (ceil(nbc / 8), nb, nsys).
__global__ __launch_bounds__(kThreads) void k_cb_gemv(int nbc, const double* __restrict__ M,
                                                     size_t msys, size_t bstride,
                                                     const double* a, const double* __restrict__ v,
                                                     double* out, size_t vsys, size_t bvstride,
                                                     Gate gate) {
  const int sys = blockIdx.z, bb = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r0 = (blockIdx.x * 4 + w) * 2;
  const double* Mb = M + (size_t)sys * msys + (size_t)bb * bstride;
  const double* vb = v + (size_t)sys * vsys + (size_t)bb * bvstride;
  double acc0 = 0.0, acc1 = 0.0;
  const bool has0 = r0 < nbc, has1 = r0 + 1 < nbc;
  for (int c = l; c < nbc; c += 64) {
    const double x = vb[c];
    if (has0) acc0 += Mb[(size_t)r0 * nbc + c] * x;
    if (has1) acc1 += Mb[(size_t)(r0 + 1) * nbc + c] * x;
  }
  acc0 = wave_sum(acc0);
  acc1 = wave_sum(acc1);
  if (l == 0) {
    const size_t ob = (size_t)sys * vsys + (size_t)bb * bvstride;
    if (has0) out[ob + r0] = a ? a[ob + r0] - acc0 : acc0;
    if (has1) out[ob + r0 + 1] = a ? a[ob + r0 + 1] - acc1 : acc1;
  }
}

// ---------------------------------------------------------------------------
// Local factors
// ---------------------------------------------------------------------------

// Level of the twisted elimination: t = 0 .. mid; at t < mid block t of the
// upper half (and block nblk - 1 - t of the lower half while t < nbot), at
// t = mid the middle block. Matrix idx of a launch: (system, subdomain) pair
// ss = idx / nh and half idx % nh; its Schur complement and then its
// inverse live in slot 2 ss + half of buffer t % 2.
struct BigLevel {
  int t, mid, nbot, nh;
};

struct MatId {
  int sys, sub, jx, jy, jz, half, ss, b;
};

__device__ inline MatId mat_id(const Geometry& g, const BigLevel& lv, int idx) {
  MatId m;
  m.ss = idx / lv.nh;
  m.half = idx - m.ss * lv.nh;
  m.sys = m.ss / g.nsub;
  m.sub = m.ss - m.sys * g.nsub;
  sub_coords(g, m.sub, m.jx, m.jy, m.jz);
  m.b = lv.t == lv.mid ? lv.mid : (m.half == 0 ? lv.t : g.nblk - 1 - lv.t);
  return m;
}

// Previous block p of term tr of matrix m, the buffer and slot of its C_p.
__device__ inline void term_of(const BigLevel& lv, const MatId& m, int tr, int& p, int& buf,
                               int& slot) {
  if (lv.t != lv.mid) {
    p = m.half == 0 ? m.b - 1 : m.b + 1;
    buf = (lv.t - 1) & 1;
    slot = 2 * m.ss + m.half;
  } else if (tr == 0) {
    p = lv.mid - 1;
    buf = (lv.mid - 1) & 1;
    slot = 2 * m.ss;
  } else {
    p = lv.mid + 1;
    buf = (lv.nbot - 1) & 1;
    slot = 2 * m.ss + 1;
  }
}

// in-layer coordinates of layer DOF o: node (x, y) (y = 0 in 2-d), component c
__device__ inline void layer_dof(const Geometry& g, int o, int& x, int& y, int& c) {
  const int n = o / g.dim;
  c = o - n * g.dim;
  if (g.dim == 3) {
    x = n % g.bn;
    y = n / g.bn;
  } else {
    x = n;
    y = 0;
  }
}

// neighbour tt of the 27 (2-d: 6) layer-coupling neighbours
__device__ inline bool nbr_of(int d, int tt, int& dx, int& dy, int& c2) {
  if (d == 3) {
    dy = tt / 9 - 1;
    dx = (tt / 3) % 3 - 1;
    c2 = tt % 3;
    return true;
  }
  dy = 0;
  dx = tt / 2 - 1;
  c2 = tt & 1;
  return tt < 6;
}

// Modulus of box-local element (ex, ey) of element layer L (between node
// layers L and L + 1): ex, ey, L in -1 .. s (the ring of the closed cell);
// zero outside the mesh and, for the Neumann matrices, outside the cell.
__device__ inline double big_modulus(const BigFactorIn& in, int sys, int jx, int jy, int jz,
                                     int ex, int ey, int L) {
  const Geometry& g = in.g;
  const int s = g.s;
  if (in.neumann) {
    if (ex < 0 || ex >= s || L < 0 || L >= s) return 0.0;
    if (g.dim == 3 && (ey < 0 || ey >= s)) return 0.0;
  }
  int gx, gy, gz;
  if (g.dim == 3) {
    gx = s * jx + ex;
    gy = s * jy + ey;
    gz = s * jz + L;
  } else {
    gx = s * jx + ex;
    gy = s * jy + L;
    gz = 0;
  }
  if (gx < 0 || gx >= g.nelx || gy < 0 || gy >= g.nely || gz < 0 || gz >= g.nelz) return 0.0;
  return in.em[(size_t)sys * g.nel + gx + (int64_t)g.nelx * (gy + (int64_t)g.nely * gz)];
}

// Stiffness between DOF o1 of node layer b1 and DOF o2 of node layer b2
// (|b1 - b2| <= 1): the sum over the elements holding both nodes.
__device__ double big_stiff(const BigFactorIn& in, const double* K0s, int sys, int jx, int jy,
                            int jz, int b1, int o1, int b2, int o2) {
  const Geometry& g = in.g;
  const int d = g.dim, nd = g.ndpe;
  int x1, y1, c1, x2, y2, c2;
  layer_dof(g, o1, x1, y1, c1);
  layer_dof(g, o2, x2, y2, c2);
  if (abs(x1 - x2) > 1 || abs(y1 - y2) > 1 || abs(b1 - b2) > 1) return 0.0;
  const int ylo = d == 3 ? max(y1, y2) - 1 : 0, yhi = d == 3 ? min(y1, y2) : 0;
  double v = 0.0;
  for (int L = max(b1, b2) - 1; L <= min(b1, b2); ++L)
    for (int ey = ylo; ey <= yhi; ++ey)
      for (int ex = max(x1, x2) - 1; ex <= min(x1, x2); ++ex) {
        const double E = big_modulus(in, sys, jx, jy, jz, ex, ey, L);
        if (E == 0.0) continue;
        const int a1 = d == 3 ? corner_of(x1 - ex, y1 - ey, b1 - L) : corner_of(x1 - ex, b1 - L, 0);
        const int a2 = d == 3 ? corner_of(x2 - ex, y2 - ey, b2 - L) : corner_of(x2 - ex, b2 - L, 0);
        v += E * K0s[(d * a1 + c1) * nd + d * a2 + c2];
      }
  return v;
}

// Matrix entry with the supports: Dirichlet A_j (supported rows and columns
// decoupled with a unit diagonal) or the scaled shifted Neumann matrix
// D^-1/2 K^N D^-1/2 + shift I (supported DOFs: fixed_diag + shift).
__device__ inline double big_entry(const BigFactorIn& in, const double* K0s, int sys, int jx,
                                   int jy, int jz, int b1, int o1, int b2, int o2, bool f1,
                                   bool f2, double s1, double s2) {
  const bool diag = b1 == b2 && o1 == o2;
  if (f1 || f2) {
    if (!diag) return 0.0;
    return in.neumann ? in.fixed_diag + in.shift : 1.0;
  }
  const double v = big_stiff(in, K0s, sys, jx, jy, jz, b1, o1, b2, o2);
  return in.neumann ? v * s1 * s2 + (diag ? in.shift : 0.0) : v;
}

__device__ inline void stage_K0(const BigFactorIn& in, double* K0s) {
  const int n = in.g.ndpe * in.g.ndpe;
  for (int i = threadIdx.x; i < n; i += blockDim.x) K0s[i] = in.K0[i];
}

// D^-1/2 of the Neumann matrices (zero on supported DOFs). grid nsub.
__global__ __launch_bounds__(kThreads) void k_big_dis(BigFactorIn in) {
  __shared__ double K0s[576];
  const Geometry& g = in.g;
  const int j = blockIdx.x;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  stage_K0(in, K0s);
  __syncthreads();
  for (int l = threadIdx.x; l < g.nloc; l += kThreads) {
    const int b = l / g.nb, o = l - (l / g.nb) * g.nb;
    const bool f = in.fixed[box_dof(g, jx, jy, jz, l)];
    const double D = f ? 0.0 : big_stiff(in, K0s, 0, jx, jy, jz, b, o, b, o);
    in.dis[(size_t)j * g.nloc + l] = (f || !(D > 0.0)) ? 0.0 : 1.0 / sqrt(D);
  }
}

// Coupling coefficients A_{b,p}[i][neighbour tt] of term tr. grid nmat.
__global__ __launch_bounds__(kThreads) void k_big_coef(BigFactorIn in, BigLevel lv, int tr,
                                                      double* __restrict__ coef) {
  __shared__ double K0s[576];
  const Geometry& g = in.g;
  const int idx = blockIdx.x;
  const MatId m = mat_id(g, lv, idx);
  int p, buf, slot;
  term_of(lv, m, tr, p, buf, slot);
  stage_K0(in, K0s);
  __syncthreads();
  const int d = g.dim, bn = g.bn, ny = d == 3 ? bn : 1;
  double* cf = coef + (size_t)idx * g.nb * 27;
  for (int e = threadIdx.x; e < g.nb * 27; e += kThreads) {
    const int i = e / 27, tt = e - (e / 27) * 27;
    int x, y, c, dx, dy, c2;
    layer_dof(g, i, x, y, c);
    double v = 0.0;
    if (nbr_of(d, tt, dx, dy, c2)) {
      const int x2 = x + dx, y2 = y + dy;
      if (x2 >= 0 && x2 < bn && y2 >= 0 && y2 < ny) {
        const int o2 = d * (x2 + bn * y2) + c2;
        const int l1 = m.b * g.nb + i, l2 = p * g.nb + o2;
        const bool f1 = in.fixed[box_dof(g, m.jx, m.jy, m.jz, l1)];
        const bool f2 = in.fixed[box_dof(g, m.jx, m.jy, m.jz, l2)];
        const double s1 = in.neumann ? in.dis[(size_t)m.sub * g.nloc + l1] : 1.0;
        const double s2 = in.neumann ? in.dis[(size_t)m.sub * g.nloc + l2] : 1.0;
        v = big_entry(in, K0s, m.sys, m.jx, m.jy, m.jz, m.b, i, p, o2, f1, f2, s1, s2);
      }
    }
    cf[e] = v;
  }
}

constexpr int kPC = 32;   // columns per workgroup of the stencil passes

__host__ __device__ inline int win_rows(const Geometry& g) { return g.dim == 3 ? 3 : 1; }
__host__ __device__ inline int row_len(const Geometry& g) { return g.dim * g.bn; }
inline size_t pass_lds_bytes(const Geometry& g) {
  return sizeof(double) * ((size_t)win_rows(g) * row_len(g) * kPC + (size_t)g.ndpe * g.ndpe +
                           (size_t)g.nb) +
         (size_t)g.nb + 16;
}

// Y = A_{b,p} X over the node rows y of layer b (3 node rows of X's layer p
// in a window), 32 columns per workgroup, X's rows read by load(row, col).
// emit(i, col, value) takes each result. The dimension is a compile-time
// constant: the neighbour terms unroll with constant offsets, and a row's
// coefficients are read together ahead of the products (same terms, same
// order of summation, exact zeros skipped as they come).
template <int D, typename Load, typename Emit>
__device__ void stencil_rows(const Geometry& g, const double* __restrict__ cf, double* Xw, int col0,
                             Load load, Emit emit) {
  constexpr int d = D, nw = D == 3 ? 3 : 1, ntt = D == 3 ? 27 : 6;
  const int bn = g.bn, rl = d * bn, ny = D == 3 ? bn : 1;
  const int t = threadIdx.x;
  auto fill = [&](int yy) {
    double* dst = Xw + (size_t)(yy % nw) * rl * kPC;
    for (int e = t; e < rl * kPC; e += kThreads) {
      const int rr = e / kPC, cc = e - (e / kPC) * kPC;
      dst[e] = load(yy * rl + rr, col0 + cc);
    }
  };
  fill(0);
  if (ny > 1) fill(1);
  __syncthreads();
  for (int y = 0; y < ny; ++y) {
    // window rows of node rows y - 1, y, y + 1 (y - 1 = -1 is never read)
    const double* wr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) wr[k] = Xw + (size_t)(((y + k - 1) % nw + nw) % nw) * rl * kPC;
    for (int e = t; e < rl * kPC; e += kThreads) {
      const int rr = e / kPC, cc = e - (e / kPC) * kPC;
      const int i = y * rl + rr;
      const int x = rr / d;
      const double* ci = cf + (size_t)i * 27;
      double cv[ntt];
#pragma unroll
      for (int tt = 0; tt < ntt; ++tt) cv[tt] = ci[tt];
      double acc = 0.0;
#pragma unroll
      for (int tt = 0; tt < ntt; ++tt) {
        int dx, dy, c2;
        nbr_of(d, tt, dx, dy, c2);
        const int x2 = x + dx, y2 = y + dy;
        if (x2 < 0 || x2 >= bn || y2 < 0 || y2 >= ny) continue;
        const double a = cv[tt];
        if (a == 0.0) continue;
        acc += a * wr[dy + 1][(d * x2 + c2) * kPC + cc];
      }
      emit(i, col0 + cc, acc);
    }
    __syncthreads();
    if (y + 2 < ny) fill(y + 2);
    __syncthreads();
  }
}

// Pass 1 of term tr: T = (A_{b,p} C_p)^T into Tb [idx][npad][npad] (row =
// column of C_p). C_p comes from the sweep's -C_p (negated here), zero past
// nb. grid (npad / kPC, nmat).
template <int D>
__global__ __launch_bounds__(kThreads) void k_big_pass1(BigFactorIn in, BigLevel lv, int tr,
                                                       const double* __restrict__ coef,
                                                       const double* __restrict__ Cb0,
                                                       const double* __restrict__ Cb1,
                                                       double* __restrict__ Tb) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* Xw = reinterpret_cast<double*>(smem);
  const Geometry& g = in.g;
  const int idx = blockIdx.y;
  const MatId m = mat_id(g, lv, idx);
  int p, buf, slot;
  term_of(lv, m, tr, p, buf, slot);
  const BigShape bs = big_shape(g);
  const size_t matE = (size_t)bs.nl * kBTE;
  const double* Cp = (buf ? Cb1 : Cb0) + (size_t)slot * matE;
  const int nb = g.nb, npad = bs.npad;
  double* Tm = Tb + (size_t)idx * npad * npad;
  stencil_rows<D>(
      g, coef + (size_t)idx * nb * 27, Xw, blockIdx.x * kPC,
      [&](int l, int col) -> double {
        if (col >= nb) return 0.0;
        const int L = l >> 6, Cc = col >> 6;
        const double v = L >= Cc ? Cp[(size_t)big_ltile(L, Cc) * kBTE + big_cofs(l & 63, col & 63)]
                                 : Cp[(size_t)big_ltile(Cc, L) * kBTE + big_cofs(col & 63, l & 63)];
        return -v;
      },
      [&](int i, int col, double v) { Tm[(size_t)col * npad + i] = v; });
}

// Pass 2 of term tr: S_b = A_bb - A_{b,p} T (first term; A_bb alone when
// has_y = 0) or S_b -= A_{b,p} T (second term), lower tiles in C layout;
// the first writes the padding rows too (unit diagonal). grid (npad / kPC, nmat).
template <int D>
__global__ __launch_bounds__(kThreads) void k_big_pass2(BigFactorIn in, BigLevel lv, int tr,
                                                       const double* __restrict__ coef,
                                                       const double* __restrict__ Tb,
                                                       double* __restrict__ Sbuf, int first,
                                                       int has_y) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Geometry& g = in.g;
  const int nw = win_rows(g), rl = row_len(g), nb = g.nb;
  double* Xw = reinterpret_cast<double*>(smem);
  double* K0s = Xw + (size_t)nw * rl * kPC;
  double* dl = K0s + g.ndpe * g.ndpe;
  uint8_t* fl = reinterpret_cast<uint8_t*>(dl + nb);
  const int idx = blockIdx.y;
  const MatId m = mat_id(g, lv, idx);
  const BigShape bs = big_shape(g);
  const size_t matE = (size_t)bs.nl * kBTE;
  const int npad = bs.npad;
  double* Sm = Sbuf + (size_t)(2 * m.ss + m.half) * matE;
  const double* Tm = Tb + (size_t)idx * npad * npad;
  stage_K0(in, K0s);
  for (int i = threadIdx.x; i < nb; i += kThreads) {
    const int l = m.b * nb + i;
    fl[i] = in.fixed[box_dof(g, m.jx, m.jy, m.jz, l)];
    dl[i] = in.neumann ? in.dis[(size_t)m.sub * g.nloc + l] : 1.0;
  }
  __syncthreads();
  const int col0 = blockIdx.x * kPC;
  auto emit = [&](int i, int j, double y) {
    if ((i >> 6) < (j >> 6)) return;
    double* dst = Sm + (size_t)big_ltile(i >> 6, j >> 6) * kBTE + big_cofs(i & 63, j & 63);
    if (j >= nb) y = 0.0;
    if (first) {
      const double a = j < nb ? big_entry(in, K0s, m.sys, m.jx, m.jy, m.jz, m.b, i, m.b, j, fl[i],
                                          fl[j], dl[i], dl[j])
                              : 0.0;
      *dst = a - (has_y ? y : 0.0);
    } else {
      *dst -= y;
    }
  };
  if (has_y) {
    stencil_rows<D>(
        g, coef + (size_t)idx * nb * 27, Xw, col0,
        [&](int l, int col) -> double { return col < nb ? Tm[(size_t)l * npad + col] : 0.0; },
        emit);
  } else {
    for (int e = threadIdx.x; e < nb * kPC; e += kThreads) {
      const int i = e / kPC, cc = e - (e / kPC) * kPC;
      emit(i, col0 + cc, 0.0);
    }
  }
  if (first) {
    for (int e = threadIdx.x; e < (npad - nb) * kPC; e += kThreads) {
      const int i = nb + e / kPC, j = col0 + e - (e / kPC) * kPC;
      if ((i >> 6) < (j >> 6)) continue;
      Sm[(size_t)big_ltile(i >> 6, j >> 6) * kBTE + big_cofs(i & 63, j & 63)] = i == j ? 1.0 : 0.0;
    }
  }
}

// Records of the level from the sweep's -C_b. Dirichlet: lower tiles, C
// layout, type T, zero past nb. grid (nl, nmat).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_big_store_dir(BigFactorIn in, BigLevel lv,
                                                           const double* __restrict__ Sbuf,
                                                           T* __restrict__ out) {
  const Geometry& g = in.g;
  const MatId m = mat_id(g, lv, blockIdx.y);
  const BigShape bs = big_shape(g);
  const int q = blockIdx.x;
  int I, J;
  tile_rc(q, I, J);
  const double* src = Sbuf + (size_t)(2 * m.ss + m.half) * bs.nl * kBTE + (size_t)q * kBTE;
  T* dst = out + ((size_t)(m.sys * g.nsub + m.sub) * g.nblk + m.b) * bs.rec_dir + (size_t)q * kBTE;
  for (int o = threadIdx.x; o < kBTE; o += kThreads) {
    int r, c;
    cdec(o, r, c);
    const bool in_ = kBT * I + r < g.nb && kBT * J + c < g.nb;
    dst[o] = in_ ? (T)(-src[o]) : (T)0;
  }
}

// Neumann records: all tiles, A layout, FP64, zero past nb. grid (ntb^2, nmat).
__global__ __launch_bounds__(kThreads) void k_big_store_neu(BigFactorIn in, BigLevel lv,
                                                           const double* __restrict__ Sbuf,
                                                           double* __restrict__ out) {
  const Geometry& g = in.g;
  const MatId m = mat_id(g, lv, blockIdx.y);
  const BigShape bs = big_shape(g);
  const int I = blockIdx.x / bs.ntb, J = blockIdx.x - (blockIdx.x / bs.ntb) * bs.ntb;
  const double* Sm = Sbuf + (size_t)(2 * m.ss + m.half) * bs.nl * kBTE;
  double* dst = out + ((size_t)m.sub * g.nblk + m.b) * bs.rec_neu + (size_t)blockIdx.x * kBTE;
  for (int o = threadIdx.x; o < kBTE; o += kThreads) {
    int r, c;
    adec(o, r, c);
    const int R = kBT * I + r, C = kBT * J + c;
    double v = 0.0;
    if (R < g.nb && C < g.nb)
      v = -(I >= J ? Sm[(size_t)big_ltile(I, J) * kBTE + big_cofs(r, c)]
                   : Sm[(size_t)big_ltile(J, I) * kBTE + big_cofs(c, r)]);
    dst[o] = v;
  }
}

// ---------------------------------------------------------------------------
// Single right-hand-side subdomain solves with the Dirichlet records
// ---------------------------------------------------------------------------

template <typename T>
__device__ inline T shfl_x(T v, int m) {
  return __shfl_xor(v, m, 64);
}

// y += C x for the symmetric C of one record (lower tiles, C layout): wave w
// takes tiles w, w + 4, ...; a tile's row products are summed over the 16
// lanes of a row group by a halving exchange (lane t ends with row sum t),
// its column products over the four row groups the same way. Partials per
// wave in yw[w][npad].
template <typename T>
__device__ void big_symv(const T* __restrict__ C, int nl, const T* xl, T* yw, int npad) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, tl = lane & 15, lq = lane >> 4;
  T* ym = yw + (size_t)w * npad;
  for (int q = w; q < nl; q += 4) {
    int I, J;
    tile_rc(q, I, J);
    const T* tile = C + (size_t)q * kBTE;
    T xj[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) xj[cb] = xl[kBT * J + 16 * cb + tl];
    T ra[16], ca[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) ca[cb] = 0;
    const bool off = I != J;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      T a[2][4][4];
#pragma unroll
      for (int rh = 0; rh < 2; ++rh)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) a[rh][cb][v] = tile[((((2 * h + rh) * 4 + cb) * 4 + v) << 6) + lane];
#pragma unroll
      for (int rh = 0; rh < 2; ++rh)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T s = 0;
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) s += a[rh][cb][v] * xj[cb];
          ra[(2 * h + rh) * 4 + v] = s;
        }
      if (off) {
#pragma unroll
        for (int rh = 0; rh < 2; ++rh)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T xi = xl[kBT * I + 16 * (2 * h + rh) + 4 * v + lq];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) ca[cb] += a[rh][cb][v] * xi;
          }
      }
    }
    // row sums: halve the 16 values over lane bits 3..0
    {
      T u8[8], u4[4], u2[2];
      const bool b3 = tl & 8, b2 = tl & 4, b1 = tl & 2, b0 = tl & 1;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const T keep = b3 ? ra[k + 8] : ra[k], send = b3 ? ra[k] : ra[k + 8];
        u8[k] = keep + shfl_x(send, 8);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const T keep = b2 ? u8[k + 4] : u8[k], send = b2 ? u8[k] : u8[k + 4];
        u4[k] = keep + shfl_x(send, 4);
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const T keep = b1 ? u4[k + 2] : u4[k], send = b1 ? u4[k] : u4[k + 2];
        u2[k] = keep + shfl_x(send, 2);
      }
      const T keep = b0 ? u2[1] : u2[0], send = b0 ? u2[0] : u2[1];
      const T rs = keep + shfl_x(send, 1);
      ym[kBT * I + 16 * (tl >> 2) + 4 * (tl & 3) + lq] += rs;
    }
    if (off) {
      const bool q1 = lq & 2, q0 = lq & 1;
      T v2[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const T keep = q1 ? ca[k + 2] : ca[k], send = q1 ? ca[k] : ca[k + 2];
        v2[k] = keep + shfl_x(send, 32);
      }
      const T keep = q0 ? v2[1] : v2[0], send = q0 ? v2[0] : v2[1];
      const T cs = keep + shfl_x(send, 16);
      ym[kBT * J + 16 * lq + tl] += cs;
    }
  }
}

// LDS of the single right-hand-side solve kernels (elements of T): K0, the
// moduli of two element layers, x [npad], the partials [4][npad], two
// vectors [npad]; then the support flags of three node layers.
__host__ __device__ inline int strip_w(const Geometry& g) {
  return g.dim == 3 ? (g.bn + 1) * (g.bn + 1) : g.bn + 1;
}
inline size_t solve_lds_bytes(const Geometry& g, size_t e) {
  const BigShape bs = big_shape(g);
  const size_t n = (size_t)g.ndpe * g.ndpe + 2 * (size_t)strip_w(g) + 7 * (size_t)bs.npad;
  return ((n * e + 15) & ~(size_t)15) + 3 * (size_t)g.nb + 16;
}

template <typename T>
struct SolveArgs {
  Geometry g;
  const double* r;
  const T* rec;
  const T* emod;
  const uint8_t* fixed;
  const double* K0;
  T* zloc;
  Gate gate;
};

template <typename T>
struct SolveLds {
  T *K0s, *E0, *E1, *x, *yw, *va, *vb;
  uint8_t* fx;
};

template <typename T>
__device__ inline SolveLds<T> solve_lds(const Geometry& g, unsigned char* smem) {
  const BigShape bs = big_shape(g);
  SolveLds<T> s;
  s.K0s = reinterpret_cast<T*>(smem);
  s.E0 = s.K0s + g.ndpe * g.ndpe;
  s.E1 = s.E0 + strip_w(g);
  s.x = s.E1 + strip_w(g);
  s.yw = s.x + bs.npad;
  s.va = s.yw + 4 * bs.npad;
  s.vb = s.va + bs.npad;
  const size_t n = (size_t)g.ndpe * g.ndpe + 2 * (size_t)strip_w(g) + 7 * (size_t)bs.npad;
  s.fx = smem + ((n * sizeof(T) + 15) & ~(size_t)15);
  return s;
}

// moduli of element layer L of box (jx, jy, jz) in the order layer_coupling reads them
template <typename T>
__device__ inline void stage_strip(const Geometry& g, const T* es, int jx, int jy, int jz, int L,
                                   T* E) {
  const int sw = strip_w(g), d = g.dim, bn = g.bn;
  for (int i = threadIdx.x; i < sw; i += kThreads) {
    const int qx = i % (bn + 1), qy = i / (bn + 1);
    const int ex = g.s * jx - 1 + qx;
    const int ey = d == 3 ? g.s * jy - 1 + qy : g.s * jy + L;
    const int ez = d == 3 ? g.s * jz + L : 0;
    const bool in = ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely && ez >= 0 && ez < g.nelz;
    E[i] = in ? es[ex + (int64_t)g.nelx * (ey + (int64_t)g.nely * ez)] : (T)0;
  }
}

template <typename T>
__device__ inline void stage_flags(const Geometry& g, const uint8_t* fixed, int jx, int jy, int jz,
                                   int b, uint8_t* f) {
  for (int o = threadIdx.x; o < g.nb; o += kThreads) f[o] = fixed[box_dof(g, jx, jy, jz, b * g.nb + o)];
}

// One block step: x = the staged right-hand side (zero past nb); out[o] =
// base[o] - C x (base != null) or C x, for o < nb; keep[o] = out masked.
template <typename T>
__device__ inline void solve_step(const Geometry& g, const T* rec, SolveLds<T>& L,
                                  const T* base, T* out, T* keep, const uint8_t* f) {
  const BigShape bs = big_shape(g);
  lds_barrier();
  big_symv(rec, bs.nl, L.x, L.yw, bs.npad);
  __syncthreads();
  for (int o = threadIdx.x; o < bs.npad; o += kThreads) {
    if (o < g.nb) {
      const T s = (L.yw[o] + L.yw[bs.npad + o]) + (L.yw[2 * bs.npad + o] + L.yw[3 * bs.npad + o]);
      const T v = base ? base[o] - s : s;
      out[o] = v;
      keep[o] = f[o] ? (T)0 : v;
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) L.yw[w * bs.npad + o] = 0;
  }
  __syncthreads();
}

// Forward pass of one half: s_b = C_b (r_b - A_{b,p} s_p) in the half's
// order (upper: b = 0 .. mid - 1; lower: b = nblk - 1 .. mid + 1).
// grid nsys * nsub * 2: (system, subdomain, half).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_big_solve_fwd(SolveArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Geometry& g = a.g;
  const int half = blockIdx.x & 1, id = blockIdx.x >> 1;
  const int sys = id / g.nsub, j = id - (id / g.nsub) * g.nsub;
  const int mid = g.nblk / 2, nbot = g.nblk - 1 - mid;
  const int len = half == 0 ? mid : nbot;
  if (len == 0 || !gate_running(a.gate, sys)) return;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  SolveLds<T> L = solve_lds<T>(g, smem);
  const BigShape bs = big_shape(g);
  for (int i = threadIdx.x; i < g.ndpe * g.ndpe; i += kThreads) L.K0s[i] = (T)a.K0[i];
  for (int i = threadIdx.x; i < 4 * bs.npad; i += kThreads) L.yw[i] = 0;
  for (int i = threadIdx.x; i < bs.npad; i += kThreads) L.x[i] = 0;
  const double* rs = a.r + (size_t)sys * g.ndof;
  const T* es = a.emod + (size_t)sys * g.nel;
  T* zs = a.zloc + (size_t)id * g.nloc;
  const T* recs = a.rec + (size_t)id * g.nblk * bs.rec_dir;
  for (int k = 0; k < len; ++k) {
    const int b = half == 0 ? k : g.nblk - 1 - k;
    // the coupling layer to the previous block: upper p = b - 1 (element
    // layer b - 1, o on its top face), lower p = b + 1 (element layer b)
    if (k > 0) stage_strip(g, es, jx, jy, jz, half == 0 ? b - 1 : b, L.E0);
    stage_flags<T>(g, a.fixed, jx, jy, jz, b, L.fx);
    __syncthreads();
    for (int o = threadIdx.x; o < g.nb; o += kThreads) {
      T v = 0;
      if (!L.fx[o]) {
        v = (T)rs[box_dof(g, jx, jy, jz, b * g.nb + o)];
        if (k > 0) v -= layer_coupling(g.dim, g.bn, L.K0s, L.E0, L.va, o, half == 0);
      }
      L.x[o] = v;
    }
    __syncthreads();
    solve_step<T>(g, recs + (size_t)b * bs.rec_dir, L, nullptr, zs + (size_t)b * g.nb, L.vb, L.fx);
    for (int o = threadIdx.x; o < g.nb; o += kThreads) L.va[o] = L.vb[o];
    __syncthreads();
  }
}

// Middle block: x_mid = C_mid (r_mid - A_{mid,mid-1} s_{mid-1} - A_{mid,mid+1} s_{mid+1}).
// grid nsys * nsub.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_big_solve_mid(SolveArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Geometry& g = a.g;
  const int id = blockIdx.x;
  const int sys = id / g.nsub, j = id - (id / g.nsub) * g.nsub;
  if (!gate_running(a.gate, sys)) return;
  const int mid = g.nblk / 2, nbot = g.nblk - 1 - mid;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  SolveLds<T> L = solve_lds<T>(g, smem);
  const BigShape bs = big_shape(g);
  for (int i = threadIdx.x; i < g.ndpe * g.ndpe; i += kThreads) L.K0s[i] = (T)a.K0[i];
  for (int i = threadIdx.x; i < 4 * bs.npad; i += kThreads) L.yw[i] = 0;
  for (int i = threadIdx.x; i < bs.npad; i += kThreads) L.x[i] = 0;
  const double* rs = a.r + (size_t)sys * g.ndof;
  const T* es = a.emod + (size_t)sys * g.nel;
  T* zs = a.zloc + (size_t)id * g.nloc;
  const T* recs = a.rec + (size_t)id * g.nblk * bs.rec_dir;
  uint8_t* fm = L.fx;              // flags of block mid
  uint8_t* fa = L.fx + g.nb;       // mid - 1
  uint8_t* fb = L.fx + 2 * g.nb;   // mid + 1
  stage_flags<T>(g, a.fixed, jx, jy, jz, mid, fm);
  if (mid >= 1) {
    stage_flags<T>(g, a.fixed, jx, jy, jz, mid - 1, fa);
    stage_strip(g, es, jx, jy, jz, mid - 1, L.E0);
  }
  if (nbot >= 1) {
    stage_flags<T>(g, a.fixed, jx, jy, jz, mid + 1, fb);
    stage_strip(g, es, jx, jy, jz, mid, L.E1);
  }
  __syncthreads();
  for (int o = threadIdx.x; o < g.nb; o += kThreads) {
    L.va[o] = (mid >= 1 && !fa[o]) ? zs[(size_t)(mid - 1) * g.nb + o] : (T)0;
    L.vb[o] = (nbot >= 1 && !fb[o]) ? zs[(size_t)(mid + 1) * g.nb + o] : (T)0;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < g.nb; o += kThreads) {
    T v = 0;
    if (!fm[o]) {
      v = (T)rs[box_dof(g, jx, jy, jz, mid * g.nb + o)];
      if (mid >= 1) v -= layer_coupling(g.dim, g.bn, L.K0s, L.E0, L.va, o, true);
      if (nbot >= 1) v -= layer_coupling(g.dim, g.bn, L.K0s, L.E1, L.vb, o, false);
    }
    L.x[o] = v;
  }
  __syncthreads();
  solve_step<T>(g, recs + (size_t)mid * bs.rec_dir, L, nullptr, zs + (size_t)mid * g.nb, L.va, fm);
}

// Backward pass of one half: x_b = s_b - C_b A_{b,q} x_q, q the block
// nearer the middle (upper: b = mid - 1 .. 0, q = b + 1, element layer b;
// lower: b = mid + 1 .. nblk - 1, q = b - 1, element layer b - 1).
// grid nsys * nsub * 2.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_big_solve_bwd(SolveArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Geometry& g = a.g;
  const int half = blockIdx.x & 1, id = blockIdx.x >> 1;
  const int sys = id / g.nsub, j = id - (id / g.nsub) * g.nsub;
  const int mid = g.nblk / 2, nbot = g.nblk - 1 - mid;
  const int len = half == 0 ? mid : nbot;
  if (len == 0 || !gate_running(a.gate, sys)) return;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  SolveLds<T> L = solve_lds<T>(g, smem);
  const BigShape bs = big_shape(g);
  for (int i = threadIdx.x; i < g.ndpe * g.ndpe; i += kThreads) L.K0s[i] = (T)a.K0[i];
  for (int i = threadIdx.x; i < 4 * bs.npad; i += kThreads) L.yw[i] = 0;
  for (int i = threadIdx.x; i < bs.npad; i += kThreads) L.x[i] = 0;
  const T* es = a.emod + (size_t)sys * g.nel;
  T* zs = a.zloc + (size_t)id * g.nloc;
  const T* recs = a.rec + (size_t)id * g.nblk * bs.rec_dir;
  uint8_t* fq = L.fx + g.nb;   // flags of block q (for the first step: mid)
  stage_flags<T>(g, a.fixed, jx, jy, jz, mid, fq);
  __syncthreads();
  for (int o = threadIdx.x; o < g.nb; o += kThreads)
    L.va[o] = fq[o] ? (T)0 : zs[(size_t)mid * g.nb + o];
  for (int k = 0; k < len; ++k) {
    const int b = half == 0 ? mid - 1 - k : mid + 1 + k;
    stage_strip(g, es, jx, jy, jz, half == 0 ? b : b - 1, L.E0);
    stage_flags<T>(g, a.fixed, jx, jy, jz, b, L.fx);
    __syncthreads();
    for (int o = threadIdx.x; o < g.nb; o += kThreads)
      L.x[o] = L.fx[o] ? (T)0 : layer_coupling(g.dim, g.bn, L.K0s, L.E0, L.va, o, half != 0);
    __syncthreads();
    T* zb = zs + (size_t)b * g.nb;
    solve_step<T>(g, recs + (size_t)b * bs.rec_dir, L, zb, zb, L.vb, L.fx);
    for (int o = threadIdx.x; o < g.nb; o += kThreads) L.va[o] = L.vb[o];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Multi right-hand-side solves with the Neumann records (eigensolver)
// ---------------------------------------------------------------------------

// Y_b = base + C_b V (base != null) or C_b V for the m <= 16 columns of V
// (Vg [npad][16], zero past nb and past m): wave w takes the tile rows I =
// w, w + 4, ...; A operands are the record's fragments, B operands V's rows.
__device__ void big_gemm16(const double* __restrict__ rec, int ntb, const double* Vg, int nb,
                           int m, const double* base, double* out) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, tl = lane & 15, lq = lane >> 4;
  for (int I = w; I < ntb; I += 4) {
    d4 acc[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = (d4){0.0, 0.0, 0.0, 0.0};
    for (int J = 0; J < ntb; ++J) {
      const double* tile = rec + ((size_t)I * ntb + J) * kBTE;
      const double* vj = Vg + (size_t)kBT * J * 16;
#pragma unroll
      for (int k0 = 0; k0 < 16; k0 += 4) {
        double a[4][4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          b[u] = vj[(4 * (k0 + u) + lq) * 16 + tl];
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) a[u][rb] = tile[((rb * 16 + k0 + u) << 6) + lane];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) acc[rb] = mfma4(a[u][rb], b[u], acc[rb]);
      }
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = kBT * I + 16 * rb + 4 * v + lq;
        if (row < nb && tl < m) {
          const double val = acc[rb][v];
          out[(size_t)row * m + tl] = base ? base[(size_t)row * m + tl] + val : val;
        }
      }
  }
}

// Right-hand side of a multi-vector step: V[o][c] = (X_b[o][c] if X) -
// sum over the couplings of block b with the blocks ps[k] (their results
// at Yp[k]); zero past nb and m. The backward step passes no X, so V = -w
// and x_b = s_b + C_b V.
__device__ void multi_rhs(const BigFactorIn& in, const double* K0s, int jx, int jy, int jz, int sub,
                          int b, const double* X, int nterm, const int* ps, const double* const* Yp,
                          int m, double* Vg, int npad) {
  const Geometry& g = in.g;
  const int d = g.dim, bn = g.bn, ny = d == 3 ? bn : 1, nb = g.nb;
  for (int o = threadIdx.x; o < npad; o += kThreads) {
    double v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = 0.0;
    if (o < nb) {
      if (X)
        for (int c = 0; c < m; ++c) v[c] = X[(size_t)o * m + c];
      const int l1 = b * nb + o;
      const bool f1 = in.fixed[box_dof(g, jx, jy, jz, l1)];
      const double s1 = in.dis[(size_t)sub * g.nloc + l1];
      int x, y, c1;
      layer_dof(g, o, x, y, c1);
      if (!f1) {
        for (int k = 0; k < nterm; ++k) {
          const int p = ps[k];
          const int ntt = d == 3 ? 27 : 6;
          for (int tt = 0; tt < ntt; ++tt) {
            int dx, dy, c2;
            nbr_of(d, tt, dx, dy, c2);
            const int x2 = x + dx, y2 = y + dy;
            if (x2 < 0 || x2 >= bn || y2 < 0 || y2 >= ny) continue;
            const int o2 = d * (x2 + bn * y2) + c2, l2 = p * nb + o2;
            if (in.fixed[box_dof(g, jx, jy, jz, l2)]) continue;
            const double a = big_stiff(in, K0s, 0, jx, jy, jz, b, o, p, o2) * s1 *
                             in.dis[(size_t)sub * g.nloc + l2];
            if (a == 0.0) continue;
            const double* yr = Yp[k] + (size_t)o2 * m;
#pragma unroll
            for (int c = 0; c < 16; ++c)
              if (c < m) v[c] -= a * yr[c];
          }
        }
      }
    }
    double* dst = Vg + (size_t)o * 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) dst[c] = v[c];
  }
}

// phase 0: forward passes (grid nsub * 2), 1: middle block (grid nsub),
// 2: backward passes (grid nsub * 2). Y receives s_b, then x_b.
__global__ __launch_bounds__(kThreads) void k_big_multi(BigFactorIn in, const double* __restrict__ rec,
                                                       int m, const double* __restrict__ X,
                                                       double* __restrict__ Y,
                                                       double* __restrict__ Vws, int phase) {
  __shared__ double K0s[576];
  const Geometry& g = in.g;
  const BigShape bs = big_shape(g);
  const int half = phase == 1 ? 0 : (blockIdx.x & 1);
  const int j = phase == 1 ? blockIdx.x : (blockIdx.x >> 1);
  const int mid = g.nblk / 2, nbot = g.nblk - 1 - mid;
  const int len = phase == 1 ? 1 : (half == 0 ? mid : nbot);
  if (len == 0) return;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  stage_K0(in, K0s);
  __syncthreads();
  const size_t rows = (size_t)g.nloc * m;
  const double* Xj = X + (size_t)j * rows;
  double* Yj = Y + (size_t)j * rows;
  double* Vg = Vws + (size_t)(2 * j + half) * bs.npad * 16;
  const double* recj = rec + (size_t)j * g.nblk * bs.rec_neu;
  const size_t bstep = (size_t)g.nb * m;
  for (int k = 0; k < len; ++k) {
    int b, ps[2], nterm = 0;
    const double* Yp[2];
    const double* Xb = nullptr;
    const double* base = nullptr;
    if (phase == 0) {
      b = half == 0 ? k : g.nblk - 1 - k;
      Xb = Xj + (size_t)b * bstep;
      if (k > 0) {
        ps[0] = half == 0 ? b - 1 : b + 1;
        Yp[0] = Yj + (size_t)ps[0] * bstep;
        nterm = 1;
      }
    } else if (phase == 1) {
      b = mid;
      Xb = Xj + (size_t)b * bstep;
      if (mid >= 1) {
        ps[nterm] = mid - 1;
        Yp[nterm++] = Yj + (size_t)(mid - 1) * bstep;
      }
      if (nbot >= 1) {
        ps[nterm] = mid + 1;
        Yp[nterm++] = Yj + (size_t)(mid + 1) * bstep;
      }
    } else {
      b = half == 0 ? mid - 1 - k : mid + 1 + k;
      ps[0] = half == 0 ? b + 1 : b - 1;
      Yp[0] = Yj + (size_t)ps[0] * bstep;
      nterm = 1;
      base = Yj + (size_t)b * bstep;
    }
    multi_rhs(in, K0s, jx, jy, jz, j, b, Xb, nterm, ps, Yp, m, Vg, bs.npad);
    __syncthreads();
    big_gemm16(recj + (size_t)b * bs.rec_neu, bs.ntb, Vg, g.nb, m, base, Yj + (size_t)b * bstep);
    __syncthreads();
  }
}

}  // namespace

const char* big_limits(const Geometry& g) {
  if (pass_lds_bytes(g) > 160 * 1024 || solve_lds_bytes(g, sizeof(double)) > 160 * 1024)
    return "subdomain node layers too large for the HBM-resident factor kernels' LDS";
  return nullptr;
}

bool local_is_big(const Geometry& g, int big_min_nb) {
  if (big_min_nb > 0 && g.nb >= big_min_nb) return true;
  if (g.nb > kMaxNb || (g.nb & 1)) return true;
  return (g.dim == 3 ? (g.bn + 1) * (g.bn + 1) : g.bn + 1) > 64;
}

void sweep_invert(double* S, size_t mstride, int nmat, int ntb, double* ws, int* flag,
                  hipStream_t st) {
  sweep_pivots(S, mstride, nmat, ntb, ntb, ws, flag, st);
}

void sweep_pivots(double* S, size_t mstride, int nmat, int ntb, int npiv, double* ws, int* flag,
                  hipStream_t st) {
  if (nmat <= 0) return;
  double* pinv = ws;
  double* Wp = pinv + (size_t)nmat * kBTE;
  double* Vp = Wp + (size_t)nmat * ntb * kBTE;
  const int nl = big_nl(ntb);
  for (int K = 0; K < npiv; ++K) {
    hipLaunchKernelGGL(k_sw_pivot, dim3(nmat), dim3(64), 0, st, S, mstride, K, pinv, flag);
    if (ntb > 1)
      hipLaunchKernelGGL(k_sw_panel, dim3(ntb, nmat), dim3(kThreads), 0, st, S, mstride, ntb, K,
                         pinv, Wp, Vp);
    hipLaunchKernelGGL(k_sw_update, dim3(nl, nmat), dim3(kThreads), 0, st, S, mstride, ntb, K, pinv,
                       Wp, Vp);
  }
}

void coarse_dense_inverse(const Geometry& g, const double* Ac, size_t astride, int nsys,
                          double* S, double* ws, double* cpk, int* flag, hipStream_t st) {
  const int ntb = big_ntb(g.nt), nl = big_nl(ntb);
  const size_t mstride = (size_t)nl * kBTE;
  hipLaunchKernelGGL(k_coarse_expand, dim3(nl, nsys), dim3(kThreads), 0, st, g, Ac, astride, S,
                     mstride);
  sweep_invert(S, mstride, nsys, ntb, ws, flag, st);
  hipLaunchKernelGGL(k_coarse_store, dim3(nl, nsys), dim3(kThreads), 0, st, g, S, mstride, nl, cpk);
}

void coarse_pack_inverse(const Geometry& g, const double* inv, int nsys, double* cpk,
                         hipStream_t st) {
  const int nl = big_nl(big_ntb(g.nt));
  hipLaunchKernelGGL(k_coarse_pack, dim3(nl, nsys), dim3(kThreads), 0, st, g, inv, nl, cpk);
}

size_t big_factor_ws_elems(const Geometry& g, int nsys) {
  const BigShape bs = big_shape(g);
  const size_t nmat = (size_t)nsys * g.nsub * 2;
  return 2 * nmat * bs.nl * kBTE               // Schur complements / inverses, two levels
         + nmat * (size_t)bs.npad * bs.npad    // pass-1 products
         + nmat * (size_t)g.nb * 27            // coupling coefficients
         + sweep_ws_elems((int)nmat, bs.ntb);
}

void coarse_band_factor(const Geometry& g, const double* Ac, size_t astride, int nsys,
                        double* cband, double* ws, int* flag, hipStream_t st) {
  const int ntb = big_ntb(g.nbc), ntb2 = 2 * ntb;
  const int nl = big_nl(ntb), nl2 = big_nl(ntb2);
  const size_t wstride = (size_t)nl2 * kBTE;
  double* W = ws;
  double* sws = W + (size_t)nsys * wstride;
  const int nblk = g.nblkc;
  hipLaunchKernelGGL(k_cb_fill, dim3(nl2, nsys), dim3(kThreads), 0, st, g, Ac, astride, 0, ntb, 0,
                     W, wstride);
  for (int b = 0; b < nblk; ++b) {
    if (b > 0)
      hipLaunchKernelGGL(k_cb_shift, dim3(nl, nsys), dim3(kThreads), 0, st, ntb, W, wstride);
    const int coupling = b + 1 < nblk;
    if (coupling) {
      hipLaunchKernelGGL(k_cb_fill, dim3(nl2, nsys), dim3(kThreads), 0, st, g, Ac, astride, b + 1,
                         ntb, 1, W, wstride);
      sweep_pivots(W, wstride, nsys, ntb2, ntb, sws, flag, st);
    } else {
      sweep_pivots(W, wstride, nsys, ntb, ntb, sws, flag, st);   // the first block's tiles alone
    }
    hipLaunchKernelGGL(k_cb_extract, dim3(coupling ? nl2 : nl, nsys), dim3(kThreads), 0, st, g, W,
                       wstride, ntb, b, coupling, cband);
  }
}

void coarse_band_solve(const Geometry& g, const double* cband, const double* yc, double* xc,
                       double* cw, int nsys, const Gate& gate, hipStream_t st) {
  const int nbc = g.nbc, nblk = g.nblkc, nt = g.nt;
  const size_t bsz = (size_t)nbc * nbc;
  const size_t msys = 3 * (size_t)nblk * bsz;
  const double* Si = cband;
  const double* Lf = cband + (size_t)nblk * bsz;
  const double* Lt = cband + 2 * (size_t)nblk * bsz;
  const unsigned gx = (unsigned)((nbc + 7) / 8);
  // forward: w_0 = r_0, w_b = r_b - L_{b,b-1} w_{b-1}
  hipMemcpy2DAsync(cw, sizeof(double) * nt, yc, sizeof(double) * nt, sizeof(double) * nbc, nsys,
                   hipMemcpyDeviceToDevice, st);
  for (int b = 1; b < nblk; ++b)
    hipLaunchKernelGGL(k_cb_gemv, dim3(gx, 1, nsys), dim3(kThreads), 0, st, nbc,
                       Lf + (size_t)b * bsz, msys, (size_t)0, yc + (size_t)b * nbc,
                       cw + (size_t)(b - 1) * nbc, cw + (size_t)b * nbc, (size_t)nt, (size_t)0,
                       gate);
  // y_b = S_b^-1 w_b for every block at once
  hipLaunchKernelGGL(k_cb_gemv, dim3(gx, nblk, nsys), dim3(kThreads), 0, st, nbc, Si, msys, bsz,
                     (const double*)nullptr, cw, xc, (size_t)nt, (size_t)nbc, gate);
  // backward: x_b = y_b - L_{b+1,b}^T x_{b+1}
  for (int b = nblk - 2; b >= 0; --b)
    hipLaunchKernelGGL(k_cb_gemv, dim3(gx, 1, nsys), dim3(kThreads), 0, st, nbc,
                       Lt + (size_t)b * bsz, msys, (size_t)0, xc + (size_t)b * nbc,
                       xc + (size_t)(b + 1) * nbc, xc + (size_t)b * nbc, (size_t)nt, (size_t)0,
                       gate);
}

namespace {
template <typename K>
void allow_lds_big(K kernel) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
}
}  // namespace

template <typename T>
void big_factor(const BigFactorIn& in, T* out, double* ws, int* flag, hipStream_t st) {
  const Geometry& g = in.g;
  const BigShape bs = big_shape(g);
  const size_t nmax = (size_t)in.nsys * g.nsub * 2;
  const size_t matE = (size_t)bs.nl * kBTE;
  double* Cb[2] = {ws, ws + nmax * matE};
  double* Tb = Cb[1] + nmax * matE;
  double* coef = Tb + nmax * (size_t)bs.npad * bs.npad;
  double* sws = coef + nmax * (size_t)g.nb * 27;
  static bool attr = false;
  if (!attr) {
    allow_lds_big(&k_big_pass1<2>);
    allow_lds_big(&k_big_pass2<2>);
    allow_lds_big(&k_big_pass1<3>);
    allow_lds_big(&k_big_pass2<3>);
    attr = true;
  }
  const bool three = g.dim == 3;
  const size_t plds = pass_lds_bytes(g);
  if (in.neumann) hipLaunchKernelGGL(k_big_dis, dim3(g.nsub), dim3(kThreads), 0, st, in);
  const int mid = g.nblk / 2, nbot = g.nblk - 1 - mid;
  const int nss = in.nsys * g.nsub;
  const int nchunk = bs.npad / kPC;
  for (int t = 0; t <= mid; ++t) {
    BigLevel lv{t, mid, nbot, (t < mid && t < nbot) ? 2 : 1};
    const int nmat = nss * lv.nh;
    double* S = Cb[t & 1];
    // terms: the previous block of each half, or both halves' last blocks
    // for the middle block
    int terms[2], nterm = 0;
    if (t != mid) {
      if (t >= 1) terms[nterm++] = 0;
    } else {
      if (mid >= 1) terms[nterm++] = 0;
      if (nbot >= 1) terms[nterm++] = 1;
    }
    if (nterm == 0) {
      if (three)
        hipLaunchKernelGGL(k_big_pass2<3>, dim3(nchunk, nmat), dim3(kThreads), plds, st, in, lv, 0,
                           coef, Tb, S, 1, 0);
      else
        hipLaunchKernelGGL(k_big_pass2<2>, dim3(nchunk, nmat), dim3(kThreads), plds, st, in, lv, 0,
                           coef, Tb, S, 1, 0);
    }
    for (int k = 0; k < nterm; ++k) {
      const int tr = terms[k];
      hipLaunchKernelGGL(k_big_coef, dim3(nmat), dim3(kThreads), 0, st, in, lv, tr, coef);
      if (three) {
        hipLaunchKernelGGL(k_big_pass1<3>, dim3(nchunk, nmat), dim3(kThreads), plds, st, in, lv,
                           tr, coef, Cb[0], Cb[1], Tb);
        hipLaunchKernelGGL(k_big_pass2<3>, dim3(nchunk, nmat), dim3(kThreads), plds, st, in, lv,
                           tr, coef, Tb, S, k == 0 ? 1 : 0, 1);
      } else {
        hipLaunchKernelGGL(k_big_pass1<2>, dim3(nchunk, nmat), dim3(kThreads), plds, st, in, lv,
                           tr, coef, Cb[0], Cb[1], Tb);
        hipLaunchKernelGGL(k_big_pass2<2>, dim3(nchunk, nmat), dim3(kThreads), plds, st, in, lv,
                           tr, coef, Tb, S, k == 0 ? 1 : 0, 1);
      }
    }
    // the matrices of this level sit in slots 2 ss + half: contiguous with
    // two halves, every second slot with one
    sweep_invert(S, (lv.nh == 2 ? 1 : 2) * matE, nmat, bs.ntb, sws, flag, st);
    if (in.neumann)
      hipLaunchKernelGGL(k_big_store_neu, dim3(bs.ntb * bs.ntb, nmat), dim3(kThreads), 0, st, in,
                         lv, S, reinterpret_cast<double*>(out));
    else
      hipLaunchKernelGGL((k_big_store_dir<T>), dim3(bs.nl, nmat), dim3(kThreads), 0, st, in, lv,
                         S, out);
  }
}

template void big_factor<double>(const BigFactorIn&, double*, double*, int*, hipStream_t);
template void big_factor<float>(const BigFactorIn&, float*, double*, int*, hipStream_t);

template <typename T>
void big_local_solves(const Geometry& g, const double* r, const T* rec, const T* emod,
                      const uint8_t* fixed, const double* K0, T* zloc, int nsys, const Gate& gate,
                      hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    allow_lds_big(&k_big_solve_fwd<T>);
    allow_lds_big(&k_big_solve_mid<T>);
    allow_lds_big(&k_big_solve_bwd<T>);
    attr = true;
  }
  SolveArgs<T> a{g, r, rec, emod, fixed, K0, zloc, gate};
  const size_t lds = solve_lds_bytes(g, sizeof(T));
  const int n = nsys * g.nsub;
  hipLaunchKernelGGL(k_big_solve_fwd<T>, dim3(2 * n), dim3(kThreads), lds, st, a);
  hipLaunchKernelGGL(k_big_solve_mid<T>, dim3(n), dim3(kThreads), lds, st, a);
  hipLaunchKernelGGL(k_big_solve_bwd<T>, dim3(2 * n), dim3(kThreads), lds, st, a);
}

template void big_local_solves<double>(const Geometry&, const double*, const double*, const double*,
                                       const uint8_t*, const double*, double*, int, const Gate&,
                                       hipStream_t);
template void big_local_solves<float>(const Geometry&, const double*, const float*, const float*,
                                      const uint8_t*, const double*, float*, int, const Gate&,
                                      hipStream_t);

void big_solve_multi(const BigFactorIn& in, const double* rec, int m, const double* X, double* Y,
                     double* ws, hipStream_t st) {
  const Geometry& g = in.g;
  hipLaunchKernelGGL(k_big_multi, dim3(2 * g.nsub), dim3(kThreads), 0, st, in, rec, m, X, Y, ws, 0);
  hipLaunchKernelGGL(k_big_multi, dim3(g.nsub), dim3(kThreads), 0, st, in, rec, m, X, Y, ws, 1);
  hipLaunchKernelGGL(k_big_multi, dim3(2 * g.nsub), dim3(kThreads), 0, st, in, rec, m, X, Y, ws, 2);
}

}  // namespace tpcg
