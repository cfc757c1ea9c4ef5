// The paper's own fine-scale solver (Sec. 2.4.2): restarted GMRES whose
// preconditioner is the MsFEM coarse solve between one symmetric
// Gauss-Seidel step before and one after it,
//   x = S(r; 0);  x += Phi K_c^-1 Phi^T (r - K x);  x = S(r; x),
// S(r; x) one node-block symmetric Gauss-Seidel step on K x = r from x in
// multicolour order (a node's colour is the parity of its grid coordinates:
// bit 0 x, bit 1 y, bit 2 z; nodes of one colour share no element, so one
// colour is one parallel launch; a step is the colours in increasing order,
// then in decreasing order). The two-level additive Schwarz preconditioner
// can take its place.
//
// GMRES is preconditioned from the left, so its residual estimate is the
// preconditioned residual, and it stops when that falls to rtol times the
// preconditioned load (the convergence measure of Sec. 3.3). The Arnoldi
// vectors are orthogonalised by classical Gram-Schmidt applied twice (two
// passes of dot products and updates over the basis, each reduced in a fixed
// order); the Hessenberg least-squares problem is solved by Givens rotations
// in a one-thread-per-system kernel. All systems of a batch share the
// Arnoldi step index; a system that converges stops (its kernels return at
// once) and its iterate is formed at the end of the cycle.
#include <algorithm>
#include <climits>
#include <cmath>

#include "tpcg_internal.h"

namespace tpcg {

namespace {

// layout of the small device arrays (doubles)
constexpr size_t kGmH = 0;                                               // [sys][col][kGmMaxVec]
constexpr size_t kGmCS = kGmH + (size_t)kMaxSys * kGmMaxRestart * kGmMaxVec;
constexpr size_t kGmSN = kGmCS + (size_t)kMaxSys * kGmMaxRestart;
constexpr size_t kGmG = kGmSN + (size_t)kMaxSys * kGmMaxRestart;        // [sys][kGmMaxVec]
constexpr size_t kGmY = kGmG + (size_t)kMaxSys * kGmMaxVec;             // [sys][kGmMaxRestart]
constexpr size_t kGmHA = kGmY + (size_t)kMaxSys * kGmMaxRestart;        // [sys][kGmMaxVec]
constexpr size_t kGmHB = kGmHA + (size_t)kMaxSys * kGmMaxVec;
constexpr size_t kGmSc = kGmHB + (size_t)kMaxSys * kGmMaxVec;           // [sys][8]
constexpr size_t kGmPart = kGmSc + (size_t)kMaxSys * 8;                 // [sys][kGmMaxVec][kMaxParts]
constexpr size_t kGmPart2 = kGmPart + (size_t)kMaxSys * kGmMaxVec * kMaxParts;   // [sys][2][kMaxParts]
// scalars per system
enum { kScBnorm = 0, kScHn = 1, kScEst = 2, kScTrue = 3, kScInv = 4 };
// ints after the gate state [kNumState][kMaxSys]: per system
enum { kGiIters = 0, kGiJcyc = 1, kGiStatus = 2, kGiZero = 3, kGiNum = 4 };

__device__ inline bool gm_active(const int* istate, int sys) {
  return istate[kStRun * kMaxSys + sys] != 0;
}

// ---------------------------------------------------------------------------
// Multicolour node-block Gauss-Seidel
// ---------------------------------------------------------------------------

// corner index -> offsets within the element (inverse of corner_of)
__device__ inline void corner_offsets(int b, int& bx, int& by, int& bz) {
  const int q = b & 3;
  bx = (q == 1 || q == 2) ? 1 : 0;
  by = q >= 2 ? 1 : 0;
  bz = b >> 2;
}

// x_n += D_n^-1 (r_n - (P K P x)_n) for every node n of `colour`, D_n the
// node's diagonal block of P K P with unit rows and columns on its fixed
// components; fixed components of x stay zero. grid (parts, nsys). The 3-d
// cycle launches it; 2-d meshes take the tiled form k_sgs_colour_q4.
template <int D>
__global__ __launch_bounds__(kThreads) void k_sgs_colour(Geometry g, const double* __restrict__ rho,
                                                         const double* __restrict__ K0, double E0,
                                                         double Emin, double penal,
                                                         const uint8_t* __restrict__ fixed,
                                                         const double* __restrict__ r,
                                                         double* __restrict__ x, int colour,
                                                         Gate gate) {
  constexpr int NE = 1 << D;
  constexpr int NDPE = D * NE;
  __shared__ double K0s[NDPE * NDPE];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  for (int i = threadIdx.x; i < NDPE * NDPE; i += kThreads) K0s[i] = K0[i];
  __syncthreads();
  const int cx = colour & 1, cy = (colour >> 1) & 1, cz = (colour >> 2) & 1;
  const int mx = (g.nnx - cx + 1) / 2, my = (g.nny - cy + 1) / 2;
  const int mz = D == 3 ? (g.nnz - cz + 1) / 2 : 1;
  const int64_t count = (int64_t)mx * my * mz;
  const double* rs = rho + (size_t)sys * g.nel;
  const double* bs = r + (size_t)sys * g.ndof;
  double* xs = x + (size_t)sys * g.ndof;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * kThreads) {
    const int ix = cx + 2 * (int)(t % mx);
    const int iy = cy + 2 * (int)((t / mx) % my);
    const int iz = D == 3 ? cz + 2 * (int)(t / ((int64_t)mx * my)) : 0;
    const int64_t n = ix + (int64_t)g.nnx * (iy + (int64_t)g.nny * iz);
    double kx[D], blk[D][D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      kx[c] = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < D; ++c2) blk[c][c2] = 0.0;
    }
    for (int e = 0; e < NE; ++e) {
      const int ox = e & 1, oy = (e >> 1) & 1, oz = (e >> 2) & 1;
      const int ex = ix - 1 + ox, ey = iy - 1 + oy, ez = D == 3 ? iz - 1 + oz : 0;
      if (ex < 0 || ex >= g.nelx || ey < 0 || ey >= g.nely) continue;
      if (D == 3 && (ez < 0 || ez >= g.nelz)) continue;
      const double E =
          simp_modulus(rs[ex + (int64_t)g.nelx * (ey + (int64_t)g.nely * ez)], E0, Emin, penal);
      const int a = corner_of(1 - ox, 1 - oy, D == 3 ? 1 - oz : 0);
      for (int b = 0; b < NE; ++b) {
        int bx, by, bz;
        corner_offsets(b, bx, by, bz);
        const int64_t m = (ex + bx) + (int64_t)g.nnx * ((ey + by) + (int64_t)g.nny * (ez + bz));
        double xm[D];
#pragma unroll
        for (int c2 = 0; c2 < D; ++c2) xm[c2] = fixed[D * m + c2] ? 0.0 : xs[D * m + c2];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          double s = 0.0;
#pragma unroll
          for (int c2 = 0; c2 < D; ++c2) s += K0s[(D * a + c) * NDPE + D * b + c2] * xm[c2];
          kx[c] += E * s;
        }
      }
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int c2 = 0; c2 < D; ++c2) blk[c][c2] += E * K0s[(D * a + c) * NDPE + D * a + c2];
    }
    bool fx[D];
    double rhs[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      fx[c] = fixed[D * n + c] != 0;
      rhs[c] = fx[c] ? 0.0 : bs[D * n + c] - kx[c];
    }
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int c2 = 0; c2 < D; ++c2)
        if (fx[c] || fx[c2]) blk[c][c2] = (c == c2) ? 1.0 : 0.0;
    // blk delta = rhs by elimination without pivoting (the block is SPD)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double piv = 1.0 / blk[k][k];
#pragma unroll
      for (int i = k + 1; i < D; ++i) {
        const double f = blk[i][k] * piv;
#pragma unroll
        for (int j = k; j < D; ++j) blk[i][j] -= f * blk[k][j];
        rhs[i] -= f * rhs[k];
      }
    }
    double dl[D];
#pragma unroll
    for (int i = D - 1; i >= 0; --i) {
      double s = rhs[i];
#pragma unroll
      for (int j = i + 1; j < D; ++j) s -= blk[i][j] * dl[j];
      dl[i] = s / blk[i][i];
    }
#pragma unroll
    for (int c = 0; c < D; ++c) xs[D * n + c] = fx[c] ? 0.0 : xs[D * n + c] + dl[c];
  }
}

// 2-d form of k_sgs_colour: the colour's nodes of a tile of kSX x kSY nodes,
// one per thread (the colour takes every second node along each axis). The
// workgroup stages the tile's one-node halo of x (node pairs as 16-byte
// loads) in LDS, so that the neighbours are read once and coalesced instead
// of gathered per node; the four moduli of a node come from global memory,
// their loads issued before the staging barrier (staging them too took LDS
// that kept fewer tiles resident). Two nodes of one colour never share an
// element, so the staged values are the current ones for every neighbour a
// node reads. The same operations in the same order as k_sgs_colour<2>.
// grid (tiles, nsys).
constexpr int kSX = 64, kSY = 16;
static_assert((kSX / 2) * (kSY / 2) == kThreads, "one colour node per thread");

__global__ __launch_bounds__(kThreads) void k_sgs_colour_q4(Geometry g, const double* __restrict__ rho,
                                                            const double* __restrict__ K0, double E0,
                                                            double Emin, double penal,
                                                            const uint8_t* __restrict__ fixed,
                                                            const double* __restrict__ r,
                                                            double* __restrict__ x, int colour,
                                                            unsigned seen, Gate gate) {
  constexpr int HX = kSX + 2, HY = kSY + 2;
  __shared__ double K0s[64];
  __shared__ __align__(16) double xh[HY * HX * 2];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  const int t = threadIdx.x;
  if (t < 64) K0s[t] = K0[t];
  const int cx = colour & 1, cy = (colour >> 1) & 1;
  const int ntx = (g.nnx + kSX - 1) / kSX;
  const int x0 = (blockIdx.x % ntx) * kSX, y0 = (blockIdx.x / ntx) * kSY;
  const double* rs = rho + (size_t)sys * g.nel;
  const double* bs = r + (size_t)sys * g.ndof;
  double* xs = x + (size_t)sys * g.ndof;
  // x is P x already: every kernel writing x leaves the supported
  // components at zero. Nodes of the colours outside `seen` are read as
  // zero (the cycle's first sweep starts from x = 0 without clearing it:
  // a colour's nodes hold values once its first launch has written them).
  for (int i = t; i < HY * HX; i += kThreads) {
    const int X = x0 - 1 + i % HX, Y = y0 - 1 + i / HX;
    double2 v = {0.0, 0.0};
    if (X >= 0 && X < g.nnx && Y >= 0 && Y < g.nny && ((seen >> ((X & 1) | ((Y & 1) << 1))) & 1u))
      v = *reinterpret_cast<const double2*>(xs + 2 * (X + (int64_t)g.nnx * Y));
    *reinterpret_cast<double2*>(xh + 2 * i) = v;
  }
  const int ix = x0 + 2 * (t % (kSX / 2)) + cx, iy = y0 + 2 * (t / (kSX / 2)) + cy;
  double Ev[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ex = ix - 1 + (e & 1), ey = iy - 1 + ((e >> 1) & 1);
    const bool in = ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely && ix < g.nnx && iy < g.nny;
    const double rv = rs[in ? ex + (int64_t)g.nelx * ey : 0];
    Ev[e] = in ? simp_modulus(rv, E0, Emin, penal) : 0.0;
  }
  __syncthreads();
  if (ix >= g.nnx || iy >= g.nny) return;
  const int64_t n = ix + (int64_t)g.nnx * iy;
  double kx[2] = {0.0, 0.0}, blk[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ox = e & 1, oy = (e >> 1) & 1;
    const int ex = ix - 1 + ox, ey = iy - 1 + oy;
    if (ex < 0 || ex >= g.nelx || ey < 0 || ey >= g.nely) continue;
    const double E = Ev[e];
    const int a = corner_of(1 - ox, 1 - oy, 0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int bx, by, bz;
      corner_offsets(b, bx, by, bz);
      const int hi = (ex + bx - x0 + 1) + HX * (ey + by - y0 + 1);
      const double xm[2] = {xh[2 * hi], xh[2 * hi + 1]};
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double s = 0.0;
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) s += K0s[(2 * a + c) * 8 + 2 * b + c2] * xm[c2];
        kx[c] += E * s;
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int c2 = 0; c2 < 2; ++c2) blk[c][c2] += E * K0s[(2 * a + c) * 8 + 2 * a + c2];
  }
  bool fx[2];
  double rhs[2];
  const double2 bv = *reinterpret_cast<const double2*>(bs + 2 * n);
  const double bn[2] = {bv.x, bv.y};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    fx[c] = fixed[2 * n + c] != 0;
    rhs[c] = fx[c] ? 0.0 : bn[c] - kx[c];
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2)
      if (fx[c] || fx[c2]) blk[c][c2] = (c == c2) ? 1.0 : 0.0;
  // the 2 x 2 block solve of k_sgs_colour
  {
    const double piv = 1.0 / blk[0][0];
    const double f = blk[1][0] * piv;
    blk[1][0] -= f * blk[0][0];
    blk[1][1] -= f * blk[0][1];
    rhs[1] -= f * rhs[0];
  }
  double dl[2];
  dl[1] = rhs[1] / blk[1][1];
  dl[0] = (rhs[0] - blk[0][1] * dl[1]) / blk[0][0];
  const int hn = (ix - x0 + 1) + HX * (iy - y0 + 1);
  *reinterpret_cast<double2*>(xs + 2 * n) =
      make_double2(fx[0] ? 0.0 : xh[2 * hn] + dl[0], fx[1] ? 0.0 : xh[2 * hn + 1] + dl[1]);
}

// x += Phi x_c (the prolongation of the coarse correction) for every
// running system; fixed components untouched. Node-parallel: each node sums
// the basis functions of the (at most 2^d) subdomains holding it.
template <int D, typename P, int KM>
__global__ __launch_bounds__(kThreads) void k_prolong_add(Geometry g, const P* __restrict__ phim,
                                                          const double* __restrict__ xc,
                                                          const uint8_t* __restrict__ fixed,
                                                          double* __restrict__ x, int nsys,
                                                          Gate gate) {
  unsigned run = 0;
  for (int sys = 0; sys < nsys; ++sys)
    if (gate_running(gate, sys)) run |= 1u << sys;
  if (!run) return;
  const int s = g.s, k = g.k;
  for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < g.nnodes;
       n += (int64_t)gridDim.x * kThreads) {
    const int ix = (int)(n % g.nnx);
    const int iy = (int)((n / g.nnx) % g.nny);
    const int iz = (int)(n / ((int64_t)g.nnx * g.nny));
    const int x0 = ix == 0 ? 0 : (ix - 1) / s, x1 = min(g.gx - 1, ix / s);
    const int y0 = iy == 0 ? 0 : (iy - 1) / s, y1 = min(g.gy - 1, iy / s);
    int z0 = 0, z1 = 0;
    if (D == 3) { z0 = iz == 0 ? 0 : (iz - 1) / s; z1 = min(g.gz - 1, iz / s); }
    double acc[kMaxSys][D];
#pragma unroll
    for (int q = 0; q < kMaxSys; ++q)
#pragma unroll
      for (int c = 0; c < D; ++c) acc[q][c] = 0.0;
    for (int jz = z0; jz <= z1; ++jz)
      for (int jy = y0; jy <= y1; ++jy)
        for (int jx = x0; jx <= x1; ++jx) {
          const int j = jx + g.gx * (jy + g.gy * jz);
          const int ln = (ix - s * jx) + g.bn * ((iy - s * jy) + g.bn * (iz - s * jz));
          const int ci = coarse_index(g, jx, jy, jz, 0);
          const P* ph = phim + (size_t)j * k * g.nloc + (size_t)D * ln;
          // modes in groups of eight, the group's loads issued together from
          // valid addresses (modes past k read mode k - 1 and are zeroed)
          for (int m0 = 0; m0 < KM; m0 += 8) {
            if (m0 >= k) break;
            double pv[8][D];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int mm = min(m0 + u, k - 1);
#pragma unroll
              for (int c = 0; c < D; ++c) pv[u][c] = (double)ph[(size_t)mm * g.nloc + c];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (m0 + u >= k)
#pragma unroll
                for (int c = 0; c < D; ++c) pv[u][c] = 0.0;
#pragma unroll
            for (int q = 0; q < kMaxSys; ++q)
              if ((run >> q) & 1u) {
                double xv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) xv[u] = xc[(size_t)q * g.nt + ci + min(m0 + u, k - 1)];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                  if (m0 + u < k)
#pragma unroll
                    for (int c = 0; c < D; ++c) acc[q][c] += pv[u][c] * xv[u];
              }
          }
        }
    if constexpr (D == 2) {
      const bool f0 = fixed[2 * n] != 0, f1 = fixed[2 * n + 1] != 0;
#pragma unroll
      for (int q = 0; q < kMaxSys; ++q)
        if ((run >> q) & 1u) {
          double2* xp = reinterpret_cast<double2*>(x + (size_t)q * g.ndof + 2 * n);
          double2 v = *xp;
          if (!f0) v.x += acc[q][0];
          if (!f1) v.y += acc[q][1];
          *xp = v;
        }
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const int64_t i = D * n + c;
        if (fixed[i]) continue;
#pragma unroll
        for (int q = 0; q < kMaxSys; ++q)
          if ((run >> q) & 1u) x[(size_t)q * g.ndof + i] += acc[q][c];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Vector kernels of the Krylov loop. Each runs (parts, nsys) workgroups; part
// p takes the entries p * 256 + t + i * parts * 256, so the partial sums of a
// launch are formed and then reduced in a fixed order.
// ---------------------------------------------------------------------------

// out = P (a - b) (b may be null) for every running system
__global__ __launch_bounds__(kThreads) void k_gm_resid(const double* __restrict__ a,
                                                       const double* __restrict__ b,
                                                       const uint8_t* __restrict__ fixed,
                                                       double* __restrict__ out, int64_t n,
                                                       Gate gate) {
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  const double* as = a + (size_t)sys * n;
  const double* bs = b ? b + (size_t)sys * n : nullptr;
  double* os = out + (size_t)sys * n;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const bool f = fixed[i] != 0;
    const double av = as[i], bv = bs ? bs[i] : 0.0;
    os[i] = f ? 0.0 : av - bv;
  }
}

__global__ __launch_bounds__(kThreads) void k_gm_zero(double* __restrict__ x, int64_t n, Gate gate) {
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  double* xs = x + (size_t)sys * n;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    xs[i] = 0.0;
}

// partials of V_i . w for i in [CH z, CH z + CH) and < nvec. V_i of system s
// at V + (i nsys + s) n; w [nsys][n]. Each partial covers the same entries in
// the same order whatever CH is (the grouping only decides which workgroup
// forms it).
template <int CH>
__global__ __launch_bounds__(kThreads) void k_gm_dots(const double* __restrict__ V, int nvec,
                                                      int nsys, const double* __restrict__ w,
                                                      double* __restrict__ part, int64_t n,
                                                      Gate gate) {
  constexpr int kGmChunk = CH;
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  const int i0 = blockIdx.z * kGmChunk;
  const int nv = min(kGmChunk, nvec - i0);
  const double* ws = w + (size_t)sys * n;
  const double* vb = V + ((size_t)i0 * nsys + sys) * n;
  const size_t vstep = (size_t)nsys * n;
  double acc[kGmChunk];
#pragma unroll
  for (int u = 0; u < kGmChunk; ++u) acc[u] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    // every load issued before the products (vectors past nv read the last
    // one; their sums are never written)
    double x[kGmChunk];
#pragma unroll
    for (int u = 0; u < kGmChunk; ++u) x[u] = vb[(size_t)min(u, nv - 1) * vstep + i];
    const double wv = ws[i];
#pragma unroll
    for (int u = 0; u < kGmChunk; ++u) acc[u] += x[u] * wv;
  }
  for (int u = 0; u < nv; ++u) {
    const double s = block_sum(acc[u], sh);
    if (threadIdx.x == 0) part[((size_t)sys * kGmMaxVec + i0 + u) * kMaxParts + blockIdx.x] = s;
  }
}

// out[sys * ostride + i] = the sum of vector i's partials, in part order. grid (nvec, nsys).
__global__ __launch_bounds__(kThreads) void k_gm_sum(const double* __restrict__ part, int np,
                                                     double* __restrict__ out, int ostride,
                                                     Gate gate) {
  __shared__ double sh[4];
  const int sys = blockIdx.y, i = blockIdx.x;
  if (!gate_running(gate, sys)) return;
  const double s = sum_parts(part + ((size_t)sys * kGmMaxVec + i) * kMaxParts, np, sh);
  if (threadIdx.x == 0) out[(size_t)sys * ostride + i] = s;
}

// w -= sum_i V_i h_i (i < nvec, in increasing i); with norm_part, the
// partials of ||w||^2 afterwards go to that system's slot 0.
__global__ __launch_bounds__(kThreads) void k_gm_orth(const double* __restrict__ V, int nvec,
                                                      int nsys, const double* __restrict__ h,
                                                      double* __restrict__ w,
                                                      double* __restrict__ norm_part, int64_t n,
                                                      Gate gate) {
  __shared__ double hs[kGmMaxVec];
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  for (int i = threadIdx.x; i < nvec; i += kThreads) hs[i] = h[(size_t)sys * kGmMaxVec + i];
  __syncthreads();
  double* ws = w + (size_t)sys * n;
  const double* vb = V + (size_t)sys * n;
  const size_t vstep = (size_t)nsys * n;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double v = ws[i];
    for (int q = 0; q < nvec; ++q) v -= vb[q * vstep + i] * hs[q];
    ws[i] = v;
    acc += v * v;
  }
  if (norm_part) {
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) norm_part[(size_t)sys * kGmMaxVec * kMaxParts + blockIdx.x] = s;
  }
}

// The first pass's update fused with the second pass's dots: w -= sum_q V_q
// h_q, then the partials of V_q . w (q < nvec), reading each basis value
// once for both. Each workgroup takes tiles of 64 consecutive entries; wave
// wv owns the vectors q = wv c + u (u < c = ceil(nvec / 4) <= C), keeps their
// values of the tile in registers, and leaves its partial sum of V_q h_q in
// LDS; after the barrier every wave forms the same updated entries (the four
// partials in a fixed order) and adds its vectors' products. Partials per
// workgroup in k_gm_dots's layout. grid (np, nsys).
template <int C>
__global__ __launch_bounds__(kThreads) void k_gm_orth_dots(const double* __restrict__ V, int nvec,
                                                           int nsys, const double* __restrict__ h,
                                                           double* __restrict__ w,
                                                           double* __restrict__ part, int64_t n,
                                                           Gate gate) {
  __shared__ double pw[2][4][64];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const int c = (nvec + 3) / 4, q0 = wv * c;
  double hq[C];
  int qi[C];
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const bool ok = u < c && q0 + u < nvec;
    hq[u] = ok ? h[(size_t)sys * kGmMaxVec + q0 + u] : 0.0;
    qi[u] = ok ? q0 + u : 0;   // a valid vector whose h is zero
  }
  double* ws = w + (size_t)sys * n;
  const double* vb = V + (size_t)sys * n;
  const size_t vstep = (size_t)nsys * n;
  double acc[C];
#pragma unroll
  for (int u = 0; u < C; ++u) acc[u] = 0.0;
  int buf = 0;
  for (int64_t i0 = (int64_t)blockIdx.x * 64; i0 < n; i0 += (int64_t)gridDim.x * 64) {
    const int64_t i = i0 + lane;
    const bool in = i < n;
    const int64_t ii = in ? i : i0;
    double x[C];
#pragma unroll
    for (int u = 0; u < C; ++u) x[u] = vb[(size_t)qi[u] * vstep + ii];
    const double wi = ws[ii];
    double p = 0.0;
#pragma unroll
    for (int u = 0; u < C; ++u) p += x[u] * hq[u];
    pw[buf][wv][lane] = p;
    __syncthreads();   // (double-buffered: the next tile writes the other half)
    const double v =
        wi - ((pw[buf][0][lane] + pw[buf][1][lane]) + (pw[buf][2][lane] + pw[buf][3][lane]));
    if (wv == 0 && in) ws[i] = v;
    const double vv = in ? v : 0.0;
#pragma unroll
    for (int u = 0; u < C; ++u) acc[u] += x[u] * vv;
    buf ^= 1;
  }
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const double sum = wave_sum(acc[u]);
    if (lane == 0 && u < c && q0 + u < nvec)
      part[((size_t)sys * kGmMaxVec + q0 + u) * kMaxParts + blockIdx.x] = sum;
  }
}

// w *= inv (per system scalar)
__global__ __launch_bounds__(kThreads) void k_gm_scale(double* __restrict__ w,
                                                       const double* __restrict__ sc, int64_t n,
                                                       Gate gate) {
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  const double f = sc[(size_t)sys * 8 + kScInv];
  double* ws = w + (size_t)sys * n;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    ws[i] *= f;
}

// Column j of the Hessenberg matrix (H[:j+1, j] = hA + hB, H[j+1, j] = ||w||),
// the earlier rotations applied to it, the new rotation, the residual
// estimate, and the stopping tests. One wave per system.
__global__ __launch_bounds__(64) void k_gm_givens(int j, double* __restrict__ w, double tol,
                                                   int maxit, int nsys, int* __restrict__ istate,
                                                   int* __restrict__ gi) {
  const int sys = blockIdx.x, lane = threadIdx.x;
  if (sys >= nsys || !gm_active(istate, sys)) return;   // uniform over the wave
  double* col = w + kGmH + ((size_t)sys * kGmMaxRestart + j) * kGmMaxVec;
  double* cs = w + kGmCS + (size_t)sys * kGmMaxRestart;
  double* sn = w + kGmSN + (size_t)sys * kGmMaxRestart;
  double* gv = w + kGmG + (size_t)sys * kGmMaxVec;
  double* sc = w + kGmSc + (size_t)sys * 8;
  const double* hA = w + kGmHA + (size_t)sys * kGmMaxVec;
  const double* hB = w + kGmHB + (size_t)sys * kGmMaxVec;
  // lane i holds the new column's entry i (i <= j < 64) and rotation i (i < j),
  // loaded together; the rotations then run in order on values passed by
  // readlane, the entry that rotation i leaves behind carried to the next
  const double hv = lane <= j ? hA[lane] + hB[lane] : 0.0;
  const double ci = lane < j ? cs[lane] : 0.0, si = lane < j ? sn[lane] : 0.0;
  // the norm's partials were summed into hA[kGmMaxVec - 1]
  const double hn = sqrt(w[kGmHA + (size_t)sys * kGmMaxVec + kGmMaxVec - 1]);
  double carry = bcast_lane(hv, 0), mine = hv;
  for (int i = 0; i < j; ++i) {
    const double a = carry, b = bcast_lane(hv, i + 1);
    const double c = bcast_lane(ci, i), s = bcast_lane(si, i);
    const double ni = c * a + s * b;
    carry = -s * a + c * b;
    if (lane == i) mine = ni;
  }
  if (lane < j) col[lane] = mine;
  if (lane != 0) return;
  sc[kScHn] = hn;
  sc[kScInv] = hn > 0.0 ? 1.0 / hn : 0.0;
  col[j] = carry;
  col[j + 1] = hn;
  const double den = hypot(col[j], col[j + 1]);
  cs[j] = col[j] / den;
  sn[j] = col[j + 1] / den;
  col[j] = den;
  col[j + 1] = 0.0;
  gv[j + 1] = -sn[j] * gv[j];
  gv[j] = cs[j] * gv[j];
  int* g = gi + kGiNum * sys;
  g[kGiIters] += 1;
  g[kGiJcyc] = j + 1;
  const double rel = fabs(gv[j + 1]) / sc[kScBnorm];
  sc[kScEst] = rel;
  int stop = 0, status = TPCG_OK;
  if (!(rel == rel) || !(den > 0.0)) { stop = 1; status = TPCG_EBREAKDOWN; }
  else if (rel <= tol || hn == 0.0) stop = 1;
  else if (g[kGiIters] >= maxit) { stop = 1; status = TPCG_ENOCONV; }
  if (stop) {
    g[kGiStatus] = status;
    istate[kStRun * kMaxSys + sys] = 0;
  }
}

// y = R^-1 g for the steps of this cycle (back substitution). One thread per system.
__global__ void k_gm_backsolve(double* __restrict__ w, int nsys, const int* __restrict__ gi) {
  const int sys = threadIdx.x;
  if (sys >= nsys) return;
  const int nj = gi[kGiNum * sys + kGiJcyc];
  const double* H = w + kGmH + (size_t)sys * kGmMaxRestart * kGmMaxVec;
  const double* gv = w + kGmG + (size_t)sys * kGmMaxVec;
  double* y = w + kGmY + (size_t)sys * kGmMaxRestart;
  for (int i = nj - 1; i >= 0; --i) {
    double s = gv[i];
    for (int k = i + 1; k < nj; ++k) s -= H[(size_t)k * kGmMaxVec + i] * y[k];
    y[i] = s / H[(size_t)i * kGmMaxVec + i];
  }
}

// x += sum_i V_i y_i over this cycle's steps (x = 0 for a zero load)
__global__ __launch_bounds__(kThreads) void k_gm_update(const double* __restrict__ V, int nsys,
                                                        const double* __restrict__ w,
                                                        const int* __restrict__ gi,
                                                        double* __restrict__ x, int64_t n) {
  __shared__ double ys[kGmMaxRestart];
  const int sys = blockIdx.y;
  const int nj = gi[kGiNum * sys + kGiJcyc];
  const bool zero = gi[kGiNum * sys + kGiZero] != 0;
  if (nj == 0 && !zero) return;
  for (int i = threadIdx.x; i < nj; i += kThreads) ys[i] = w[kGmY + (size_t)sys * kGmMaxRestart + i];
  __syncthreads();
  double* xs = x + (size_t)sys * n;
  const double* vb = V + (size_t)sys * n;
  const size_t vstep = (size_t)nsys * n;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    if (zero) {
      xs[i] = 0.0;
      continue;
    }
    double v = 0.0;
    for (int q = 0; q < nj; ++q) v += vb[q * vstep + i] * ys[q];
    xs[i] += v;
  }
}

__global__ void k_gm_reset(int nsys, int* __restrict__ istate, int* __restrict__ gi) {
  const int sys = threadIdx.x;
  if (sys >= kMaxSys) return;
  for (int s = 0; s < kNumState; ++s) istate[s * kMaxSys + sys] = 0;
  istate[kStRun * kMaxSys + sys] = sys < nsys ? 1 : 0;
  for (int q = 0; q < kGiNum; ++q) gi[kGiNum * sys + q] = 0;
}

// beta = ||v0|| from the partials in slot 0. mode 0: the preconditioned load
// norm (zero: the solution is zero and the system stops). mode 1: a new
// cycle: stop if beta <= tol * the load norm or maxit is spent, else
// g = beta e_1 and v0 /= beta. grid (nsys), 256 threads.
__global__ __launch_bounds__(kThreads) void k_gm_begin(int mode, int np, double* __restrict__ w,
                                                       double tol, int maxit, int* __restrict__ istate,
                                                       int* __restrict__ gi) {
  __shared__ double sh[4];
  const int sys = blockIdx.x;
  int* g = gi + kGiNum * sys;
  double* sc = w + kGmSc + (size_t)sys * 8;
  if (mode == 1 && threadIdx.x == 0) g[kGiJcyc] = 0;
  if (!gm_active(istate, sys)) return;
  const double s = sum_parts(w + kGmPart + (size_t)sys * kGmMaxVec * kMaxParts, np, sh);
  const double beta = sqrt(s);
  if (mode == 0) {
    if (threadIdx.x == 0) {
      sc[kScBnorm] = beta;
      sc[kScEst] = 0.0;
      if (!(beta > 0.0)) {
        g[kGiZero] = 1;
        g[kGiStatus] = beta == 0.0 ? TPCG_OK : TPCG_EBREAKDOWN;
        istate[kStRun * kMaxSys + sys] = 0;
      }
    }
    return;
  }
  const double rel = beta / sc[kScBnorm];
  __syncthreads();
  if (rel <= tol || g[kGiIters] >= maxit || !(rel == rel)) {
    if (threadIdx.x == 0) {
      sc[kScEst] = rel;
      g[kGiStatus] = !(rel == rel) ? TPCG_EBREAKDOWN : (rel <= tol ? TPCG_OK : TPCG_ENOCONV);
      istate[kStRun * kMaxSys + sys] = 0;
    }
    return;
  }
  double* gv = w + kGmG + (size_t)sys * kGmMaxVec;
  for (int i = threadIdx.x; i < kGmMaxVec; i += kThreads) gv[i] = i == 0 ? beta : 0.0;
  if (threadIdx.x == 0) sc[kScInv] = 1.0 / beta;
}

// partials of ||P (f - q)||^2 and ||P f||^2
__global__ __launch_bounds__(kThreads) void k_gm_true_parts(const double* __restrict__ f,
                                                            const double* __restrict__ q,
                                                            const uint8_t* __restrict__ fixed,
                                                            double* __restrict__ part2,
                                                            int64_t n) {
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  const double* fs = f + (size_t)sys * n;
  const double* qs = q + (size_t)sys * n;
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    if (fixed[i]) continue;
    const double r = fs[i] - qs[i];
    a += r * r;
    b += fs[i] * fs[i];
  }
  const double sa = block_sum(a, sh);
  const double sb = block_sum(b, sh);
  if (threadIdx.x == 0) {
    part2[((size_t)sys * 2 + 0) * kMaxParts + blockIdx.x] = sa;
    part2[((size_t)sys * 2 + 1) * kMaxParts + blockIdx.x] = sb;
  }
}

// out[4 sys ..] = {iterations, status, estimate, true relative residual}
__global__ __launch_bounds__(kThreads) void k_gm_final(const double* __restrict__ w, int np,
                                                       const int* __restrict__ gi,
                                                       double* __restrict__ out) {
  __shared__ double sh[4];
  const int sys = blockIdx.x;
  const double* part2 = w + kGmPart2;
  const double a = sum_parts(part2 + ((size_t)sys * 2 + 0) * kMaxParts, np, sh);
  const double b = sum_parts(part2 + ((size_t)sys * 2 + 1) * kMaxParts, np, sh);
  if (threadIdx.x == 0) {
    out[4 * sys + 0] = gi[kGiNum * sys + kGiIters];
    out[4 * sys + 1] = gi[kGiNum * sys + kGiStatus];
    out[4 * sys + 2] = w[kGmSc + (size_t)sys * 8 + kScEst];
    out[4 * sys + 3] = b > 0.0 ? sqrt(a / b) : 0.0;
  }
}

__global__ void k_gm_poll(const int* __restrict__ istate, int* __restrict__ out) {
  const int sys = threadIdx.x;
  if (sys < kMaxSys) out[sys] = istate[kStRun * kMaxSys + sys];
}

int vec_parts(const Geometry& g) {
  const int64_t b = (g.ndof + 4 * kThreads - 1) / (4 * kThreads);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxParts));
}

void launch_dots(const Handle& h, int chunk, const double* V, int nv, int nsys, const double* w,
                 double* part, int np, const Gate& gate, hipStream_t st) {
  const int64_t n = h.g.ndof;
#define TPCG_DOTS(CH)                                                                          \
  hipLaunchKernelGGL(k_gm_dots<CH>, dim3(np, nsys, (nv + CH - 1) / CH), dim3(kThreads), 0, st, \
                     V, nv, nsys, w, part, n, gate)
  if (chunk == 4) TPCG_DOTS(4);
  else if (chunk == 16) TPCG_DOTS(16);
  else TPCG_DOTS(8);
#undef TPCG_DOTS
}

// the first pass's update and the second pass's dots in one launch (nv <= 64)
void launch_orth_dots(const double* V, int nv, int nsys, const double* hv, double* w, double* part,
                      int64_t n, int np, const Gate& gate, hipStream_t st) {
  static_assert(kGmMaxRestart <= 64, "four waves of at most 16 vectors");
  const int c = (nv + 3) / 4;
#define TPCG_OD(C)                                                                    \
  hipLaunchKernelGGL(k_gm_orth_dots<C>, dim3(np, nsys), dim3(kThreads), 0, st, V, nv, \
                     nsys, hv, w, part, n, gate)
  if (c <= 2) TPCG_OD(2);
  else if (c <= 4) TPCG_OD(4);
  else if (c <= 8) TPCG_OD(8);
  else TPCG_OD(16);
#undef TPCG_OD
}

}  // namespace

double gmres_time_dots(Handle& h, int nsys, int nv, int chunk) {
  const int np = vec_parts(h.g);
  Gate all{};
  all.parts = h.parts;
  all.istate = h.gm_i;
  all.rr_slot = kPartRR0;
  all.maxit = INT_MAX;
  all.enabled = 0;
  hipStream_t st = h.stream;
  const double* V = h.gm_V;
  const double* w = h.gm_V + (size_t)nv * nsys * h.g.ndof;   // vector nv of the basis
  launch_dots(h, chunk, V, nv, nsys, w, h.gm_w + kGmPart, np, all, st);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) hipEventDestroy(a);
    (void)hipGetLastError();
    return -1.0;
  }
  hipEventRecord(a, st);
  constexpr int kReps = 3;
  for (int r = 0; r < kReps; ++r)
    launch_dots(h, chunk, V, nv, nsys, w, h.gm_w + kGmPart, np, all, st);
  hipEventRecord(b, st);
  hipEventSynchronize(b);
  float ms = -1.0f;
  hipEventElapsedTime(&ms, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms > 0.0f ? ms / kReps : -1.0;
}

size_t gmres_small_elems() {
  return kGmPart2 + (size_t)kMaxSys * 2 * kMaxParts;
}

// xout = B rin with the MsFEM cycle for every running system. Uses h.q and
// h.z as work vectors (rin and xout must be neither).
void launch_msfem_cycle(Handle& h, const double* rho, const double* rin, double* xout, int nsys,
                        const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  const tpcg_problem& pr = h.prob;
  const dim3 vgrid(vec_parts(g), nsys);
  const int nc = 1 << g.dim;
  auto colour = [&](int c, unsigned seen) {
    const int64_t cnt = (int64_t)((g.nnx + 1) / 2) * ((g.nny + 1) / 2) * (g.dim == 3 ? (g.nnz + 1) / 2 : 1);
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((cnt + kThreads - 1) / kThreads, 4096)),
                    nsys);
    if (g.dim == 2) {
      const unsigned ntile = (unsigned)(((g.nnx + kSX - 1) / kSX) * ((g.nny + kSY - 1) / kSY));
      hipLaunchKernelGGL(k_sgs_colour_q4, dim3(ntile, nsys), dim3(kThreads), 0, st, g, rho, h.K0,
                         pr.E0, pr.Emin, pr.penal, h.fixed, rin, xout, c, seen, gate);
    } else
      hipLaunchKernelGGL(k_sgs_colour<3>, grid, dim3(kThreads), 0, st, g, rho, h.K0, pr.E0,
                         pr.Emin, pr.penal, h.fixed, rin, xout, c, gate);
  };
  // the colours up, then down; the last colour is not solved twice in a
  // row: its block equations hold after the first solve (its nodes share
  // no element), so a second one would change x by rounding only
  // (from zero: in 2-d the first sweep reads the colours not yet written as
  // zero instead of clearing x first)
  auto sgs_step = [&](bool from_zero) {
    for (int c = 0; c < nc; ++c) colour(c, from_zero ? (1u << c) - 1u : 0xfu);
    for (int c = nc - 2; c >= 0; --c) colour(c, 0xfu);
  };
  if (g.dim != 2) hipLaunchKernelGGL(k_gm_zero, vgrid, dim3(kThreads), 0, st, xout, g.ndof, gate);
  sgs_step(true);
  launch_apply_K(h, rho, xout, h.q, nsys, -1, gate, st);
  hipLaunchKernelGGL(k_gm_resid, vgrid, dim3(kThreads), 0, st, rin, h.q, h.fixed, h.z, g.ndof,
                     gate);
  launch_coarse_only(h, h.z, nsys, gate, st);
  const dim3 ngrid(parts_for(g.nnodes));
#define TPCG_PROLONG(D, P, KM)                                                                 \
  hipLaunchKernelGGL((k_prolong_add<D, P, KM>), ngrid, dim3(kThreads), 0, st, g,               \
                     reinterpret_cast<const P*>(h.phim), h.xc, h.fixed, xout, nsys, gate)
  if (g.dim == 2) {
    if (h.mixed) TPCG_PROLONG(2, float, kMaxK);
    else TPCG_PROLONG(2, double, kMaxK);
  } else {
    if (h.mixed) TPCG_PROLONG(3, float, kMaxK);
    else TPCG_PROLONG(3, double, kMaxK);
  }
#undef TPCG_PROLONG
  sgs_step(false);
}

int gmres_solve(Handle& h, const double* rho, const double* f, double* u, int nsys, double rtol,
                int maxit, int m, int precond, double* hout) {
  const Geometry& g = h.g;
  hipStream_t st = h.stream;
  const int64_t n = g.ndof;
  const int np = vec_parts(g);
  const dim3 vgrid(np, nsys);
  double* w = h.gm_w;
  int* istate = h.gm_i;
  int* gi = h.gm_i + kNumState * kMaxSys;
  Gate run{};
  run.parts = h.parts;
  run.istate = istate;
  run.np = 0;
  run.rr_slot = kPartRR0;
  run.it = 0;
  run.maxit = INT_MAX;
  run.tol2 = 0.0;
  run.enabled = 1;
  run.test = 0;
  run.itbase = nullptr;
  auto V = [&](int i) { return h.gm_V + (size_t)i * nsys * n; };
  auto apply_B = [&](const double* rin, double* xout) {
    if (precond == TPCG_PC_MSFEM_SGS) launch_msfem_cycle(h, rho, rin, xout, nsys, run, st);
    else launch_precond(h, rin, xout, nsys, run, kPartAux, -2, 0, st);
  };
  auto norm_into_slot0 = [&](const double* v) {
    launch_dots(h, h.gm_chunk, v, 1, nsys, v, w + kGmPart, np, run, st);
  };
  hipLaunchKernelGGL(k_gm_reset, dim3(1), dim3(64), 0, st, nsys, istate, gi);
  // the preconditioned load and its norm
  hipLaunchKernelGGL(k_gm_resid, vgrid, dim3(kThreads), 0, st, f, nullptr, h.fixed, h.r, n, run);
  apply_B(h.r, V(0));
  norm_into_slot0(V(0));
  hipLaunchKernelGGL(k_gm_begin, dim3(nsys), dim3(kThreads), 0, st, 0, np, w, rtol, maxit, istate,
                     gi);
  int total = 0;
  int* hp = h.gm_host;
  for (;;) {
    // a new cycle: v0 = B P (f - K u) / beta
    launch_apply_K(h, rho, u, h.p, nsys, -1, run, st);
    hipLaunchKernelGGL(k_gm_resid, vgrid, dim3(kThreads), 0, st, f, h.p, h.fixed, h.r, n, run);
    apply_B(h.r, V(0));
    norm_into_slot0(V(0));
    hipLaunchKernelGGL(k_gm_begin, dim3(nsys), dim3(kThreads), 0, st, 1, np, w, rtol, maxit,
                       istate, gi);
    hipLaunchKernelGGL(k_gm_scale, vgrid, dim3(kThreads), 0, st, V(0), w + kGmSc, n, run);
    int j = 0;
    for (; j < m && total < maxit; ++j, ++total) {
      double* wj = V(j + 1);
      launch_apply_K(h, rho, V(j), h.p, nsys, -1, run, st);
      apply_B(h.p, wj);
      const int nv = j + 1;
      // classical Gram-Schmidt, twice
      launch_dots(h, h.gm_chunk, V(0), nv, nsys, wj, w + kGmPart, np, run, st);
      hipLaunchKernelGGL(k_gm_sum, dim3(nv, nsys), dim3(kThreads), 0, st, w + kGmPart, np,
                         w + kGmHA, kGmMaxVec, run);
      launch_orth_dots(V(0), nv, nsys, w + kGmHA, wj, w + kGmPart, n, np, run, st);
      hipLaunchKernelGGL(k_gm_sum, dim3(nv, nsys), dim3(kThreads), 0, st, w + kGmPart, np,
                         w + kGmHB, kGmMaxVec, run);
      hipLaunchKernelGGL(k_gm_orth, vgrid, dim3(kThreads), 0, st, V(0), nv, nsys, w + kGmHB, wj,
                         w + kGmPart, n, run);
      // ||w||^2 into the last slot of hA (the hA values of this step are
      // read by the rotation kernel below before anything overwrites them)
      hipLaunchKernelGGL(k_gm_sum, dim3(1, nsys), dim3(kThreads), 0, st, w + kGmPart, np,
                         w + kGmHA + kGmMaxVec - 1, kGmMaxVec, run);
      hipLaunchKernelGGL(k_gm_givens, dim3(nsys), dim3(64), 0, st, j, w, rtol, maxit, nsys, istate,
                         gi);
      hipLaunchKernelGGL(k_gm_scale, vgrid, dim3(kThreads), 0, st, wj, w + kGmSc, n, run);
      // poll the running flags one step behind the launches
      const int slot = total & 1;
      hipLaunchKernelGGL(k_gm_poll, dim3(1), dim3(64), 0, st, istate, h.gm_flags + slot * kMaxSys);
      hipMemcpyAsync(hp + slot * kMaxSys, h.gm_flags + slot * kMaxSys, sizeof(int) * kMaxSys,
                     hipMemcpyDeviceToHost, st);
      hipEventRecord(h.gm_ev[slot], st);
      if (j > 0) {
        const int prev = slot ^ 1;
        if (hipEventSynchronize(h.gm_ev[prev]) != hipSuccess) return TPCG_EHIP;
        int any = 0;
        for (int s = 0; s < nsys; ++s) any |= hp[prev * kMaxSys + s];
        if (!any) {
          ++j;
          ++total;
          break;
        }
      }
    }
    hipLaunchKernelGGL(k_gm_backsolve, dim3(1), dim3(64), 0, st, w, nsys, gi);
    hipLaunchKernelGGL(k_gm_update, vgrid, dim3(kThreads), 0, st, V(0), nsys, w, gi, u, n);
    // the cycle's end: stop when no system runs
    hipLaunchKernelGGL(k_gm_poll, dim3(1), dim3(64), 0, st, istate, h.gm_flags);
    hipMemcpyAsync(hp, h.gm_flags, sizeof(int) * kMaxSys, hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess) return TPCG_EHIP;
    int any = 0;
    for (int s = 0; s < nsys; ++s) any |= hp[s];
    if (!any || total >= maxit) break;
  }
  // every system has stopped (converged, maxit spent inside the rotation
  // kernel or at a cycle's start, or broken down): the true residual
  Gate all = run;
  all.enabled = 0;
  launch_apply_K(h, rho, u, h.p, nsys, -1, all, st);
  hipLaunchKernelGGL(k_gm_true_parts, vgrid, dim3(kThreads), 0, st, f, h.p, h.fixed, w + kGmPart2,
                     n);
  hipLaunchKernelGGL(k_gm_final, dim3(nsys), dim3(kThreads), 0, st, w, np, gi, h.gm_out);
  hipMemcpyAsync(hout, h.gm_out, sizeof(double) * 4 * nsys, hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) return TPCG_EHIP;
  return TPCG_OK;
}

}  // namespace tpcg
