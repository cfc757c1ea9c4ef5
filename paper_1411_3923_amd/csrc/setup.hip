// Construction of the two-level preconditioner (Sec. 2.4, Sec. 3.2, Sec. 5.3):
//   1. Neumann matrices K_j^N of each cell (its own elements only, physical
//      supports kept) of the representative system, scaled to
//      S_j = D^-1/2 K_j^N D^-1/2 with D = diag(K_j^N), and factored shifted.
//   2. The k smallest eigenpairs of S_j by shift-invert block subspace
//      iteration (Cholesky QR applied twice) and a final Rayleigh-Ritz step;
//      psi = D^-1/2 x solves K_j^N psi = lambda D psi.
//   3. Phi_j = chi_j psi_j with chi_j(n) = 1 / (subdomains containing n).
//   4. Per system: W_j = K Phi_j on the cell grown by one node layer, the
//      Galerkin blocks Phi_l^T W_j of K_c = Phi^T K Phi, the coarse factor and,
//      for moderate coarse dimensions, the dense K_c^-1.
//   5. Per system: local Dirichlet matrices A_j (principal submatrices of
//      the supported K on the closed-cell DOFs) and their twisted
//      factors (eliminated from both ends towards the middle block), on the
//      second stream, concurrently with 4.
// All factors are block-tridiagonal Cholesky factors (see btri.h).
#include <algorithm>
#include <vector>

#include "big.h"
#include "btri.h"

namespace tpcg {

namespace {

constexpr double kFixedDiag = 1.0e3;   // decoupled supported DOFs of S_j sit far above its spectrum

struct MatParams {
  double E0, Emin, penal, shift;
};

// Deterministic start vectors of the subspace iteration.
__device__ inline double hash_uniform(uint64_t a) {
  // splitmix64 finaliser, mapped to [-1, 1)
  a += 0x9E3779B97F4A7C15ull;
  a = (a ^ (a >> 30)) * 0xBF58476D1CE4E5B9ull;
  a = (a ^ (a >> 27)) * 0x94D049BB133111EBull;
  a ^= a >> 31;
  return (double)(a >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(kThreads) void k_eig_init(Geometry g, double* __restrict__ X,
                                                      const double* __restrict__ dis, int m) {
  const int j = blockIdx.x, jp = phys_sub(g, j);   // start vectors seeded by the subdomain
  for (int e = threadIdx.x; e < g.nloc * m; e += kThreads) {
    const int l = e / m;
    const double v = dis[(size_t)j * g.nloc + l] > 0.0
                         ? hash_uniform(((uint64_t)jp * g.nloc + l) * 64 + (e - l * m))
                         : 0.0;
    X[(size_t)j * g.nloc * m + e] = v;
  }
}

// Orthonormalise the columns of X[j] (nloc x m, row-major, m <= 16) in place
// by Cholesky QR applied twice: G = X^T X (on the matrix cores:
// v_mfma_f64_16x16x4f64 with both operands read from X, four waves over
// interleaved row chunks, partial tiles summed in LDS), G + s I = R^T R with a
// tiny shift s = 1e-14 trace(G) that keeps the factorisation defined when X is
// ill-conditioned, then X <- X R^-1. The second pass restores orthogonality to
// working accuracy. Supported DOFs are zeroed first.
typedef double dv4 __attribute__((ext_vector_type(4)));

// part[w] = this wave's share of A^T B (16 x 16 tile, row-major, m <= 16
// columns, rows of A and B with stride m): wave w takes the 4-row chunks
// 4 (w + 4 i); eight chunks are loaded before their products are formed.
// Sum part[0..3] for the product.
__device__ void gram_waves(const double* __restrict__ A, const double* __restrict__ B, int n,
                           int m, double (*part)[256]) {
  constexpr int kU = 8;
  const int t = threadIdx.x, wv = t >> 6, l = t & 63, li = l & 15, lq = l >> 4;
  dv4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 4 * wv; k0 < n; k0 += 16 * kU) {
    double va[kU], vb[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int row = k0 + 16 * u + lq;
      const bool in = row < n && li < m;
      va[u] = in ? A[(size_t)row * m + li] : 0.0;
      vb[u] = in ? B[(size_t)row * m + li] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], vb[u], acc, 0, 0, 0);
  }
  for (int q = 0; q < 4; ++q) part[wv][(4 * q + lq) * 16 + li] = acc[q];
}

__global__ __launch_bounds__(kThreads) void k_eig_cholqr(Geometry g, double* __restrict__ X,
                                                        const double* __restrict__ dis, int m) {
  __shared__ double part[4][256];
  __shared__ double U[16 * 16];
  __shared__ double ip[16];   // inverse pivots 1 / U[b][b]
  const int j = blockIdx.x;
  double* Xj = X + (size_t)j * g.nloc * m;
  const double* dj = dis + (size_t)j * g.nloc;
  const int t = threadIdx.x;
  for (int r = t; r < g.nloc; r += kThreads)
    if (dj[r] == 0.0)
      for (int c = 0; c < m; ++c) Xj[(size_t)r * m + c] = 0.0;
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    gram_waves(Xj, Xj, g.nloc, m, part);   // G = X^T X
    __syncthreads();
    // G + shift I = U^T U (upper Cholesky) on wave 0, lane b holding column
    // b of U; every pivot and every entry of a pivot's column reaches the
    // other lanes by readlane
    if (t < 64) {
      const int b = t;
      double g[16], u[16];
#pragma unroll
      for (int a = 0; a < 16; ++a) {
        const int e = a * 16 + (b & 15);
        g[a] = (a < m && b < m) ? (part[0][e] + part[1][e]) + (part[2][e] + part[3][e]) : 0.0;
        u[a] = 0.0;
      }
      double tr = 0.0;   // trace of G: lane a holds G[a][a] in g[a]
#pragma unroll
      for (int a = 0; a < 16; ++a)
        if (a < m) tr += bcast_lane(g[a], a);
      const double shift = 1e-14 * tr;
#pragma unroll
      for (int a = 0; a < 16; ++a) {
        if (a < m) {
          double sd = g[a] + shift;   // meaningful in lane a
#pragma unroll
          for (int c = 0; c < a; ++c) sd -= u[c] * u[c];
          const double d = bcast_lane(sd > 0.0 ? sqrt(sd) : 1.0, a);
          double v = g[a];   // G[a][b] in lane b
#pragma unroll
          for (int c = 0; c < a; ++c) v -= bcast_lane(u[c], a) * u[c];
          u[a] = b == a ? d : (b > a ? v / d : 0.0);
        }
      }
      if (b < 16)
#pragma unroll
        for (int a = 0; a < 16; ++a) U[a * 16 + b] = u[a];
      if (b < 16) ip[b] = b < m ? 1.0 / u[b] : 0.0;
    }
    __syncthreads();
    // X <- X U^-1 row by row: forward substitution x_new U = x
    for (int r = t; r < g.nloc; r += kThreads) {
      int oz = 0;   // opaque: U is read per row, not held in registers
      asm volatile("" : "+v"(oz));
      const double* Uv = U + oz;
      const double* iv = ip + oz;
      double x[kMaxSub];
#pragma unroll
      for (int c = 0; c < kMaxSub; ++c) x[c] = c < m ? Xj[(size_t)r * m + c] : 0.0;
#pragma unroll
      for (int b = 0; b < kMaxSub; ++b) {
        if (b < m) {
          double v = x[b];
#pragma unroll
          for (int a = 0; a < b; ++a) v -= x[a] * Uv[a * 16 + b];
          x[b] = v * iv[b];
          Xj[(size_t)r * m + b] = x[b];
        }
      }
    }
    __syncthreads();
  }
}

// Y = (L L^T)^-1 X for every subdomain, m right-hand sides (FP64).
// D = g.dim as a constant, so that the accumulators are indexed statically
// and stay in registers
template <int D>
__global__ __launch_bounds__(kThreads) void k_neumann_apply(Geometry g, const double* __restrict__ rho,
                                                           const double* __restrict__ K0,
                                                           const double* __restrict__ dis,
                                                           const double* __restrict__ X,
                                                           double* __restrict__ Y, int m,
                                                           MatParams mp) {
  __shared__ double K0s[576];
  const int j = blockIdx.x, jp = phys_sub(g, j);
  const int jx = jp % g.gx, jy = (jp / g.gx) % g.gy, jz = jp / (g.gx * g.gy);
  constexpr int d = D, nd = D == 3 ? 24 : 8;
  for (int i = threadIdx.x; i < nd * nd; i += kThreads) K0s[i] = K0[i];
  __syncthreads();
  const double* dj = dis + (size_t)j * g.nloc;
  const double* Xj = X + (size_t)j * g.nloc * m;
  double* Yj = Y + (size_t)j * g.nloc * m;
  for (int ln = threadIdx.x; ln < g.nbox; ln += kThreads) {
    const int lx = ln % g.bn, ly = (ln / g.bn) % g.bn, lz = ln / (g.bn * g.bn);
    double acc[D][kMaxSub];
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int r = 0; r < kMaxSub; ++r) acc[c][r] = 0.0;
    constexpr int na = D == 3 ? 8 : 4;
    for (int a = 0; a < na; ++a) {
      const int dx = (a & 3) == 1 || (a & 3) == 2, dy = (a & 3) >= 2, dz = a >= 4;
      const int ex = lx - dx, ey = ly - dy, ez = lz - dz;   // cell-local element
      if (ex < 0 || ex >= g.s || ey < 0 || ey >= g.s || (d == 3 && (ez < 0 || ez >= g.s))) continue;
      const int gex = g.s * jx + ex, gey = g.s * jy + ey, gez = g.s * jz + ez;
      const double E = simp_modulus(
          rho[gex + (int64_t)g.nelx * (gey + (int64_t)g.nely * gez)], mp.E0, mp.Emin, mp.penal);
      for (int bnode = 0; bnode < na; ++bnode) {
        const int bx = ex + ((bnode & 3) == 1 || (bnode & 3) == 2);
        const int by = ey + ((bnode & 3) >= 2);
        const int bz = ez + (bnode >= 4);
        const int lb = bx + g.bn * (by + g.bn * bz);
        for (int cc = 0; cc < d; ++cc) {
          const int l2 = d * lb + cc;
          const double s2 = dj[l2];
          if (s2 == 0.0) continue;
          double xv[kMaxSub];
#pragma unroll
          for (int r = 0; r < kMaxSub; ++r) xv[r] = r < m ? Xj[(size_t)l2 * m + r] : 0.0;
#pragma unroll
          for (int c = 0; c < D; ++c) {
            const double kv = E * K0s[(d * a + c) * nd + d * bnode + cc] * s2;
#pragma unroll
            for (int r = 0; r < kMaxSub; ++r) acc[c][r] += kv * xv[r];
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const int l = d * ln + c;
      const double s1 = dj[l];
#pragma unroll
      for (int r = 0; r < kMaxSub; ++r)
        if (r < m) Yj[(size_t)l * m + r] = s1 * acc[c][r];
    }
  }
}

__device__ inline int axis_mult(int i, int s, int nel) {
  return (i % s == 0 && i > 0 && i < nel) ? 2 : 1;
}

// ---------------------------------------------------------------------------
// Distinct cells (Sec. 2.4: equal agglomerates of a periodic microstructure
// share their local eigenproblem). The eigenproblem of subdomain j is fixed
// by the densities of its cell's elements (cell order) and the supports of
// its box DOFs (box order).
// ---------------------------------------------------------------------------

__device__ inline uint64_t mix64(uint64_t x) {   // the splitmix64 finaliser
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__device__ inline int64_t cell_element(const Geometry& g, int jx, int jy, int jz, int q) {
  const int ex = q % g.s, ey = (q / g.s) % g.s, ez = g.dim == 3 ? q / (g.s * g.s) : 0;
  return (int64_t)(g.s * jx + ex) +
         (int64_t)g.nelx * ((g.s * jy + ey) + (int64_t)g.nely * (g.s * jz + ez));
}

// sig[j] = the sum mod 2^64 of a mix of every (position, value) of the
// subdomain's data: equal data, equal signature (candidates are then
// compared exactly)
__global__ __launch_bounds__(kThreads) void k_cell_sig(Geometry g, const double* __restrict__ rho,
                                                      const uint8_t* __restrict__ fixed,
                                                      unsigned long long* __restrict__ sig) {
  __shared__ unsigned long long part[kThreads];
  const int j = blockIdx.x;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  const int ncell = g.dim == 3 ? g.s * g.s * g.s : g.s * g.s;
  uint64_t acc = 0;
  for (int q = threadIdx.x; q < ncell; q += kThreads) {
    uint64_t bits;
    const double v = rho[cell_element(g, jx, jy, jz, q)];
    memcpy(&bits, &v, sizeof(bits));
    acc += mix64(bits ^ mix64((uint64_t)q));
  }
  for (int l = threadIdx.x; l < g.nloc; l += kThreads)
    acc += mix64(((uint64_t)fixed[box_dof(g, jx, jy, jz, l)] + 1) ^ mix64((uint64_t)(ncell + l)));
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t s = 0;
    for (int i = 0; i < kThreads; ++i) s += part[i];
    sig[j] = s;
  }
}

// flag[i] = 1 if subdomain pairs[2 i] differs from pairs[2 i + 1] anywhere
__global__ __launch_bounds__(kThreads) void k_cell_same(Geometry g, const double* __restrict__ rho,
                                                       const uint8_t* __restrict__ fixed,
                                                       const int* __restrict__ pairs,
                                                       int* __restrict__ flag) {
  const int i = blockIdx.x;
  const int a = pairs[2 * i], b = pairs[2 * i + 1];
  int ax, ay, az, bx, by, bz;
  sub_coords(g, a, ax, ay, az);
  sub_coords(g, b, bx, by, bz);
  const int ncell = g.dim == 3 ? g.s * g.s * g.s : g.s * g.s;
  int diff = 0;
  for (int q = threadIdx.x; q < ncell; q += kThreads) {
    const double va = rho[cell_element(g, ax, ay, az, q)], vb = rho[cell_element(g, bx, by, bz, q)];
    uint64_t ua, ub;
    memcpy(&ua, &va, sizeof(ua));
    memcpy(&ub, &vb, sizeof(ub));
    diff |= ua != ub;
  }
  for (int l = threadIdx.x; l < g.nloc; l += kThreads)
    diff |= fixed[box_dof(g, ax, ay, az, l)] != fixed[box_dof(g, bx, by, bz, l)];
  diff = __syncthreads_or(diff);
  if (threadIdx.x == 0) flag[i] = diff;
}

__device__ inline int box_mult(const Geometry& g, int jx, int jy, int jz, int ln) {
  const int lx = ln % g.bn, ly = (ln / g.bn) % g.bn, lz = ln / (g.bn * g.bn);
  int mult = axis_mult(g.s * jx + lx, g.s, g.nelx) * axis_mult(g.s * jy + ly, g.s, g.nely);
  if (g.dim == 3) mult *= axis_mult(g.s * jz + lz, g.s, g.nelz);
  return mult;
}

// The eigenpairs of each duplicate pairs[2 i] from its representative
// pairs[2 i + 1]: Phi with the duplicate's partition-of-unity weights (the
// weights are 1/2^n, so the rescaling is exact), Ritz values, residuals and
// the count of vectors in use.
__global__ __launch_bounds__(kThreads) void k_dedup_scatter(Geometry g, const int* __restrict__ pairs,
                                                           double* __restrict__ phi,
                                                           double* __restrict__ lam,
                                                           double* __restrict__ eres,
                                                           int* __restrict__ kj, int m) {
  const int i = blockIdx.x;
  const int a = pairs[2 * i], b = pairs[2 * i + 1];
  int ax, ay, az, bx, by, bz;
  sub_coords(g, a, ax, ay, az);
  sub_coords(g, b, bx, by, bz);
  const int k = g.k;
  for (int e = threadIdx.x; e < g.nloc * k; e += kThreads) {
    const int l = e / k;
    const int ln = l / g.dim;
    const double f = (double)box_mult(g, bx, by, bz, ln);
    const double w = (double)box_mult(g, ax, ay, az, ln);
    phi[(size_t)a * g.nloc * k + e] = phi[(size_t)b * g.nloc * k + e] * f / w;
  }
  for (int r = threadIdx.x; r < m; r += kThreads) {
    lam[(size_t)a * m + r] = lam[(size_t)b * m + r];
    eres[(size_t)a * m + r] = eres[(size_t)b * m + r];
  }
  if (threadIdx.x == 0) kj[a] = kj[b];
}

// Rayleigh-Ritz on span(X) with SX = S X: H = X^T S X, H = Q Theta Q^T
// (cyclic Jacobi), Ritz vectors X Q in ascending order; writes the Ritz
// values, the residual norms ||S x - theta x|| and Phi_j = chi D^-1/2 (X Q)[:, :k].
// With thr > 0 only the Ritz vectors of Ritz values below thr (at most k)
// are kept; the other columns of Phi_j are zero and kj[j] counts the kept.
__global__ __launch_bounds__(kThreads) void k_eig_rr(Geometry g, const double* __restrict__ X,
                                                    const double* __restrict__ SX,
                                                    const double* __restrict__ dis, int m,
                                                    double* __restrict__ lam,
                                                    double* __restrict__ eres,
                                                    double* __restrict__ phi, double thr,
                                                    int* __restrict__ kj) {
  __shared__ double sh[4];
  __shared__ double part[4][256];
  __shared__ double H[kMaxSub * kMaxSub];
  __shared__ double Qm[kMaxSub * kMaxSub];
  __shared__ double Qo[kMaxSub * kMaxSub];   // Ritz vectors in ascending order, zero-padded
  __shared__ double th[kMaxSub];
  __shared__ int ord[kMaxSub];
  __shared__ int done;
  const int t = threadIdx.x;
  const int j = blockIdx.x;            // work arrays: launch index
  const int jp = phys_sub(g, j);       // outputs and geometry: the subdomain
  const int jx = jp % g.gx, jy = (jp / g.gx) % g.gy, jz = jp / (g.gx * g.gy);
  const double* Xj = X + (size_t)j * g.nloc * m;
  const double* Sj = SX + (size_t)j * g.nloc * m;
  gram_waves(Xj, Sj, g.nloc, m, part);   // H = X^T S X
  __syncthreads();
  if (t < kMaxSub * kMaxSub) {
    const int a = t >> 4, b = t & 15;
    const double h = a < m && b < m ? (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]) : 0.0;
    const double ht = a < m && b < m ? (part[0][b * 16 + a] + part[1][b * 16 + a]) +
                                           (part[2][b * 16 + a] + part[3][b * 16 + a])
                                     : 0.0;
    H[t] = 0.5 * (h + ht);   // symmetrised
    Qm[t] = a == b ? 1.0 : 0.0;
  }
  __syncthreads();
  // cyclic Jacobi: for each pair (p, q) every thread forms the rotation, and
  // thread r < m applies it to entry r of columns p, q of H and Q, then to
  // entry r of rows p, q of H
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (t == 0) {
      double off = 0.0, dia = 0.0;
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
          const double v = H[a * kMaxSub + b];
          if (a == b) dia += v * v; else off += v * v;
        }
      done = off <= 1e-30 * dia;
    }
    __syncthreads();
    if (done) break;
    for (int p = 0; p < m; ++p)
      for (int qq = p + 1; qq < m; ++qq) {
        const double apq = H[p * kMaxSub + qq];
        const double app = H[p * kMaxSub + p], aqq = H[qq * kMaxSub + qq];
        __syncthreads();   // every thread has read the pivot entries
        if (apq == 0.0) continue;
        const double tau = (aqq - app) / (2.0 * apq);
        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + tt * tt), sn = tt * c;
        if (t < m) {
          const double hp = H[t * kMaxSub + p], hq = H[t * kMaxSub + qq];
          H[t * kMaxSub + p] = c * hp - sn * hq;
          H[t * kMaxSub + qq] = sn * hp + c * hq;
          const double qp = Qm[t * kMaxSub + p], qv = Qm[t * kMaxSub + qq];
          Qm[t * kMaxSub + p] = c * qp - sn * qv;
          Qm[t * kMaxSub + qq] = sn * qp + c * qv;
        }
        __syncthreads();
        if (t < m) {
          const double hp = H[p * kMaxSub + t], hq = H[qq * kMaxSub + t];
          H[p * kMaxSub + t] = c * hp - sn * hq;
          H[qq * kMaxSub + t] = sn * hp + c * hq;
        }
        __syncthreads();
      }
  }
  if (t == 0) {
    for (int a = 0; a < m; ++a) { th[a] = H[a * kMaxSub + a]; ord[a] = a; }
    for (int a = 1; a < m; ++a) {          // insertion sort, ascending
      const int o = ord[a];
      int b = a - 1;
      while (b >= 0 && th[ord[b]] > th[o]) { ord[b + 1] = ord[b]; --b; }
      ord[b + 1] = o;
    }
  }
  __syncthreads();
  if (t < kMaxSub * kMaxSub) {
    const int r = t >> 4, i = t & 15;
    Qo[t] = r < m && i < m ? Qm[r * kMaxSub + ord[i]] : 0.0;
  }
  __syncthreads();
  // modes in use: the first kuse in ascending order
  int kuse = g.k;
  if (thr > 0.0) {
    kuse = 0;
    while (kuse < g.k && th[ord[kuse]] < thr) ++kuse;
  }
  if (t == 0) kj[jp] = kuse;
  // residuals and the basis
  double racc[kMaxSub];
#pragma unroll
  for (int i = 0; i < kMaxSub; ++i) racc[i] = 0.0;
  const int k = g.k;
  for (int l = t; l < g.nloc; l += kThreads) {
    // an opaque offset keeps the compiler from hoisting all of Qo out of the
    // loop into registers
    int oz = 0;
    asm volatile("" : "+v"(oz));
    const double* Qv = Qo + oz;
    double xr[kMaxSub], sr[kMaxSub];
#pragma unroll
    for (int r = 0; r < kMaxSub; ++r) {
      xr[r] = r < m ? Xj[(size_t)l * m + r] : 0.0;
      sr[r] = r < m ? Sj[(size_t)l * m + r] : 0.0;
    }
    const double sd = dis[(size_t)j * g.nloc + l];
    const int ln = l / g.dim;
    const int lx = ln % g.bn, ly = (ln / g.bn) % g.bn, lz = ln / (g.bn * g.bn);
    int mult = axis_mult(g.s * jx + lx, g.s, g.nelx) * axis_mult(g.s * jy + ly, g.s, g.nely);
    if (g.dim == 3) mult *= axis_mult(g.s * jz + lz, g.s, g.nelz);
    const double chi = 1.0 / mult;
#pragma unroll 1
    for (int i = 0; i < m; ++i) {
      double xv = 0.0, sv = 0.0;
#pragma unroll
      for (int r = 0; r < kMaxSub; ++r) {
        const double qv = Qv[r * kMaxSub + i];
        xv += xr[r] * qv;
        sv += sr[r] * qv;
      }
      const double res = sv - th[ord[i]] * xv;
#pragma unroll
      for (int ii = 0; ii < kMaxSub; ++ii) racc[ii] += ii == i ? res * res : 0.0;
      if (i < k) phi[((size_t)jp * g.nloc + l) * k + i] = i < kuse ? chi * sd * xv : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < kMaxSub; ++i) {
    if (i >= m) break;
    const double v = block_sum(racc[i], sh);
    if (t == 0) {
      lam[(size_t)jp * m + i] = th[ord[i]];
      eres[(size_t)jp * m + i] = sqrt(v);
    }
  }
}

// ---------------------------------------------------------------------------
// Galerkin coarse matrix
// ---------------------------------------------------------------------------

// W[j][en][c][m] = (K Phi_j) at the node en of the cell grown by one node
// layer (zero outside the mesh).
// blockIdx.y = system: moduli at rho + y nel, W at W + y wstride
template <int D, int KM>
__global__ __launch_bounds__(kThreads) void k_coarse_W(Geometry g, const double* __restrict__ rho,
                                                      const double* __restrict__ K0,
                                                      const uint8_t* __restrict__ fixed,
                                                      const double* __restrict__ phi,
                                                      double* __restrict__ W, size_t wstride,
                                                      MatParams mp) {
  __shared__ double K0s[576];
  const int j = blockIdx.x, jp = phys_sub(g, j);
  const int jx = jp % g.gx, jy = (jp / g.gx) % g.gy, jz = jp / (g.gx * g.gy);
  constexpr int d = D, nd = D == 3 ? 24 : 8;
  const int k = g.k;
  for (int i = threadIdx.x; i < nd * nd; i += kThreads) K0s[i] = K0[i];
  __syncthreads();
  const double* ph = phi + (size_t)j * g.nloc * k;
  double* Wj = W + blockIdx.y * wstride + (size_t)j * g.nebox * d * k;
  rho += (size_t)blockIdx.y * g.nel;
  const int e = g.ebn;
  for (int en = threadIdx.x; en < g.nebox; en += kThreads) {
    const int ex_ = en % e, ey_ = (en / e) % e, ez_ = en / (e * e);
    const int nx = g.s * jx - 1 + ex_, ny = g.s * jy - 1 + ey_;
    const int nz = d == 3 ? g.s * jz - 1 + ez_ : 0;
    double acc[D][KM];
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int mm = 0; mm < KM; ++mm) acc[c][mm] = 0.0;
    const bool in_mesh = nx >= 0 && nx < g.nnx && ny >= 0 && ny < g.nny && nz >= 0 && nz < g.nnz;
    if (in_mesh) {
      constexpr int na = D == 3 ? 8 : 4;
      for (int a = 0; a < na; ++a) {
        const int dx = (a & 3) == 1 || (a & 3) == 2, dy = (a & 3) >= 2, dz = a >= 4;
        const int elx = nx - dx, ely = ny - dy, elz = nz - dz;
        if (elx < 0 || elx >= g.nelx || ely < 0 || ely >= g.nely) continue;
        if (d == 3 && (elz < 0 || elz >= g.nelz)) continue;
        const double E = simp_modulus(rho[elx + (int64_t)g.nelx * (ely + (int64_t)g.nely * elz)],
                                      mp.E0, mp.Emin, mp.penal);
        for (int bnode = 0; bnode < na; ++bnode) {
          const int bx = elx + ((bnode & 3) == 1 || (bnode & 3) == 2);
          const int by = ely + ((bnode & 3) >= 2);
          const int bz = elz + (bnode >= 4);
          const int lx = bx - g.s * jx, ly = by - g.s * jy, lz = d == 3 ? bz - g.s * jz : 0;
          if (lx < 0 || lx > g.s || ly < 0 || ly > g.s || lz < 0 || lz > (d == 3 ? g.s : 0)) continue;
          const int lb = lx + g.bn * (ly + g.bn * lz);
          for (int cc = 0; cc < d; ++cc) {
            const double* pv = ph + ((size_t)d * lb + cc) * k;
            double pvv[KM];
#pragma unroll
            for (int mm = 0; mm < KM; ++mm) pvv[mm] = mm < k ? pv[mm] : 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
              const double kv = E * K0s[(d * a + c) * nd + d * bnode + cc];
#pragma unroll
              for (int mm = 0; mm < KM; ++mm) acc[c][mm] += kv * pvv[mm];
            }
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const bool fx = in_mesh && fixed[(int64_t)d * (nx + (int64_t)g.nnx * (ny + (int64_t)g.nny * nz)) + c];
#pragma unroll
      for (int mm = 0; mm < KM; ++mm)
        if (mm < k) Wj[((size_t)en * d + c) * k + mm] = (in_mesh && !fx) ? acc[c][mm] : 0.0;
    }
  }
}

// Blocks Phi_l^T W_j of K_c for every neighbour l of j whose coarse block is
// j's block or the next one (the lower part of the block-tridiagonal
// storage), every k <= 16, on the FP64 matrix cores. Unused modes (zero
// columns of Phi, threshold mode) get a unit diagonal, so that K_c stays
// nonsingular and their coarse unknowns stay zero. The rows of the product are the (node, component) pairs of box l
// inside the extended box of j; lane (i, kk) of a wave feeds mode i of row
// kk of a four-row chunk of Phi_l and of W_j to v_mfma_f64_16x16x4f64, the
// four waves taking every fourth chunk and eight chunks' loads issued ahead
// of their products. grid.x = nsub * 3^d, grid.y = system.
template <int D>
__global__ __launch_bounds__(kThreads) void k_coarse_assemble_mma(Geometry g,
                                                                  const double* __restrict__ phi,
                                                                  const double* __restrict__ W,
                                                                  size_t wstride,
                                                                  double* __restrict__ cf,
                                                                  size_t cstride,
                                                                  const int* __restrict__ kj) {
  __shared__ double part[kThreads / 64][256];
  constexpr int d = D, nnb = D == 3 ? 27 : 9;
  const int j = blockIdx.x / nnb;
  const int o = blockIdx.x - j * nnb;
  const int jx = j % g.gx, jy = (j / g.gx) % g.gy, jz = j / (g.gx * g.gy);
  const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = D == 3 ? o / 9 - 1 : 0;
  const int lx = jx + ox, ly = jy + oy, lz = jz + oz;
  if (lx < 0 || lx >= g.gx || ly < 0 || ly >= g.gy || lz < 0 || lz >= g.gz) return;
  const int k = g.k;
  const int Rb = coarse_index(g, lx, ly, lz, 0), Cb = coarse_index(g, jx, jy, jz, 0);
  const int rblk = Rb / g.nbc, cblk = Cb / g.nbc;
  int slot;
  if (rblk == cblk) slot = 0;
  else if (rblk == cblk + 1) slot = 1;
  else return;
  const int l = lx + g.gx * (ly + g.gy * lz);
  const double* pl = phi + (size_t)l * g.nloc * k;
  const double* Wj = W + blockIdx.y * wstride + (size_t)j * g.nebox * d * k;
  const int x0 = max(g.s * lx, g.s * jx - 1), x1 = min(g.s * lx + g.s, g.s * jx + g.s + 1);
  const int y0 = max(g.s * ly, g.s * jy - 1), y1 = min(g.s * ly + g.s, g.s * jy + g.s + 1);
  int z0 = 0, z1 = 0;
  if (D == 3) { z0 = max(g.s * lz, g.s * jz - 1); z1 = min(g.s * lz + g.s, g.s * jz + g.s + 1); }
  const int nxr = x1 - x0 + 1, nyr = y1 - y0 + 1, nzr = z1 - z0 + 1;
  const int nrow = nxr * nyr * nzr * d;
  double* blk = cf + blockIdx.y * cstride + ((size_t)rblk * 2 + slot) * g.nbc * g.nbc;
  const int rin = Rb - rblk * g.nbc, cin = Cb - cblk * g.nbc;
  const int e = g.ebn;
  const int t = threadIdx.x, wv = t >> 6, ln = t & 63, li = ln & 15, lq = ln >> 4;
  constexpr int kU = 8;
  dv4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = 4 * wv; r0 < nrow; r0 += 16 * kU) {
    double va[kU], vb[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int row = r0 + 16 * u + lq;
      va[u] = vb[u] = 0.0;
      if (row < nrow && li < k) {
        const int idx = row / d, c = row - (row / d) * d;
        const int nx = x0 + idx % nxr, ny = y0 + (idx / nxr) % nyr, nz = z0 + idx / (nxr * nyr);
        const int lb = (nx - g.s * lx) + g.bn * ((ny - g.s * ly) + g.bn * (nz - g.s * lz));
        const int eb = (nx - g.s * jx + 1) +
                       e * ((ny - g.s * jy + 1) + e * (D == 3 ? nz - g.s * jz + 1 : 0));
        va[u] = pl[((size_t)d * lb + c) * k + li];
        vb[u] = Wj[((size_t)eb * d + c) * k + li];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], vb[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) part[wv][(4 * q + lq) * 16 + li] = acc[q];
  __syncthreads();
  if (t < 256) {
    const int a = t >> 4, b = t & 15;
    if (a < k && b < k) {
      double v = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
      if (l == j && a == b && a >= kj[j]) v = 1.0;
      blk[(size_t)(rin + a) * g.nbc + cin + b] = v;
    }
  }
}

// moduli E_e of the systems the local factors are built from
template <typename T>
__global__ void k_moduli(const double* __restrict__ rho, T* __restrict__ out, int64_t n,
                         double E0, double Emin, double penal) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    out[i] = (T)simp_modulus(rho[i], E0, Emin, penal);
}

// mode-major copy of Phi for the iteration kernels: out[j][m][l] = phi[j][l][m]
template <typename T>
__global__ void k_phi_modes(Geometry g, const double* __restrict__ phi, T* __restrict__ out) {
  const int64_t n = (int64_t)g.nsub * g.nloc * g.k;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const int64_t j = i / ((int64_t)g.k * g.nloc);
    const int rem = (int)(i - j * g.k * g.nloc);
    const int m = rem / g.nloc, l = rem - (rem / g.nloc) * g.nloc;
    out[i] = (T)phi[((size_t)j * g.nloc + l) * g.k + m];
  }
}

template <typename T>
T* dalloc(size_t n, int& err) {
  void* p = nullptr;
  if (n == 0) n = 1;
  if (!device_alloc(&p, n * sizeof(T))) { err = TPCG_ENOMEM; return nullptr; }
  return reinterpret_cast<T*>(p);
}

}  // namespace

size_t build_ws_elems(const tpcg_problem& pr, const Geometry& g, int big, int msub) {
  const size_t nsl = (size_t)g.nsub * g.nloc;
  const size_t m = msub;
  size_t eig;
  if (big) {
    // Neumann records, D^-1/2, two subspace blocks, the representative
    // moduli, then the factorisation's work arrays (later the multi-vector
    // solves')
    const BigShape bs = big_shape(g);
    eig = (size_t)g.nsub * g.nblk * bs.rec_neu + nsl * (1 + 2 * m) + (size_t)g.nel +
          std::max(big_factor_ws_elems(g, 1), big_multi_ws_elems(g));
  } else {
    eig = (size_t)g.nsub * g.nblk * g.bstride + nsl * (1 + 2 * m);
  }
  const size_t wsz = (size_t)g.nsub * g.nebox * g.dim * g.k;
  const size_t asm_coarse = (size_t)g.nblkc * 2 * g.nbc * g.nbc;
  size_t coarse = (wsz + asm_coarse) * pr.nsys_max;
  if (g.nt <= g.dense_max && !g.cband) coarse += coarse_dense_ws_elems(g, pr.nsys_max);
  if (g.cband) coarse += coarse_band_ws_elems(g, pr.nsys_max);
  if (big) coarse += big_factor_ws_elems(g, pr.nsys_max);
  return std::max(eig, coarse);
}

// Distinct cells of the representative design: signatures on the GPU, groups
// on the host, every candidate duplicate compared exactly on the GPU (a
// signature collision leaves the cell its own representative). Writes the
// representatives to h.submap_d (ascending) and the (duplicate,
// representative) pairs to h.dedup_pairs. Synchronises the stream.
int distinct_cells(Handle& h, const double* rrep, hipStream_t st, int& nrep, int& npairs) {
  const Geometry& g = h.g;
  hipLaunchKernelGGL(k_cell_sig, dim3(g.nsub), dim3(kThreads), 0, st, g, rrep, h.fixed, h.cell_sig);
  std::vector<unsigned long long> sig(g.nsub);
  hipMemcpyAsync(sig.data(), h.cell_sig, sizeof(unsigned long long) * g.nsub,
                 hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) return TPCG_EHIP;
  std::vector<int> rep(g.nsub);
  {
    std::vector<std::pair<unsigned long long, int>> order(g.nsub);
    for (int j = 0; j < g.nsub; ++j) order[j] = {sig[j], j};
    std::sort(order.begin(), order.end());
    for (size_t i = 0; i < order.size(); ++i)
      rep[order[i].second] = (i > 0 && order[i].first == order[i - 1].first)
                                 ? rep[order[i - 1].second]
                                 : order[i].second;   // the lowest index of the group
  }
  std::vector<int> pairs;
  for (int j = 0; j < g.nsub; ++j)
    if (rep[j] != j) {
      pairs.push_back(j);
      pairs.push_back(rep[j]);
    }
  if (!pairs.empty()) {
    const int np = (int)pairs.size() / 2;
    hipMemcpyAsync(h.dedup_pairs, pairs.data(), sizeof(int) * pairs.size(), hipMemcpyHostToDevice,
                   st);
    hipLaunchKernelGGL(k_cell_same, dim3(np), dim3(kThreads), 0, st, g, rrep, h.fixed,
                       h.dedup_pairs, h.dedup_flag);
    std::vector<int> differ(np);
    hipMemcpyAsync(differ.data(), h.dedup_flag, sizeof(int) * np, hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess) return TPCG_EHIP;
    for (int i = 0; i < np; ++i)
      if (differ[i]) rep[pairs[2 * i]] = pairs[2 * i];
  }
  std::vector<int> reps;
  pairs.clear();
  for (int j = 0; j < g.nsub; ++j) {
    if (rep[j] == j) {
      reps.push_back(j);
    } else {
      pairs.push_back(j);
      pairs.push_back(rep[j]);
    }
  }
  nrep = (int)reps.size();
  npairs = (int)pairs.size() / 2;
  hipMemcpyAsync(h.submap_d, reps.data(), sizeof(int) * reps.size(), hipMemcpyHostToDevice, st);
  if (npairs > 0)
    hipMemcpyAsync(h.dedup_pairs, pairs.data(), sizeof(int) * pairs.size(), hipMemcpyHostToDevice,
                   st);
  // the host vectors must outlive the copies
  return hipStreamSynchronize(st) == hipSuccess ? TPCG_OK : TPCG_EHIP;
}

int build_preconditioner(Handle& h, const double* rho, int nsys, int rep, int with_basis) {
  const Geometry& g = h.g;
  hipStream_t st = h.stream;
  const tpcg_problem& pr = h.prob;
  int err = TPCG_OK;
  const BtriShape lsh = local_shape(g), csh = coarse_shape(g);
  const size_t asm_coarse = (size_t)g.nblkc * 2 * g.nbc * g.nbc;
  const size_t rec = h.big ? (size_t)g.nsub * g.nblk * big_shape(g).rec_neu
                           : (size_t)g.nsub * g.nblk * g.bstride;
  const int m = h.msub;
  const int iters = pr.eig_iters > 0 ? pr.eig_iters : 6;
  MatParams mp{pr.E0, pr.Emin, pr.penal, pr.eig_shift != 0.0 ? pr.eig_shift : 1.0e-5};

  // work arrays of the build, kept by the handle from one build to the next:
  // the eigensolver's (Neumann factor, scaling, two subspace blocks), then the
  // coarse assembly's. The factorisations compute their matrices block by
  // block from the element moduli, so no assembled matrix is stored.
  const size_t nsl = (size_t)g.nsub * g.nloc;
  const size_t wsz = (size_t)g.nsub * g.nebox * g.dim * g.k;
  const size_t need = build_ws_elems(pr, g, h.big, m);
  if (h.build_elems < need) {
    if (h.build_ws) hipFree(h.build_ws);
    h.build_ws = nullptr;
    h.build_elems = 0;
    h.build_ws = dalloc<double>(need, err);
    h.build_elems = h.build_ws ? need : 0;
    if (err) { h.err = "out of device memory for the preconditioner build"; return err; }
  }
  hipMemsetAsync(h.dflag, 0, 4 * sizeof(int), st);
  StencilIn si{};
  si.g = g;
  si.fixed = h.fixed;
  si.K0 = h.K0;
  si.E0 = pr.E0;
  si.Emin = pr.Emin;
  si.penal = pr.penal;
  si.shift = mp.shift;
  si.fixed_diag = kFixedDiag;
  // --- 1-3: spectral basis from system `rep` (kept as it is when !with_basis) ---
  if (with_basis) {
  double* nfac = h.build_ws;
  double* dis = nfac + rec;
  double* X = dis + nsl;
  double* Y = X + nsl * m;
  const double* rrep = rho + (size_t)rep * g.nel;
  BigFactorIn nin{};
  double* fws = Y + nsl * m + g.nel;   // big path: factorisation, then multi-vector work arrays
  // distinct cells only (the on-chip path): the eigen phase runs on the
  // representatives, launch index c working on subdomain submap[c], and the
  // duplicates take their eigenpairs afterwards
  Geometry ge = g;
  int nrep = g.nsub, npairs = 0;
  if (pr.dedup && !h.big) {
    const int rc = distinct_cells(h, rrep, st, nrep, npairs);
    if (rc != TPCG_OK) return rc;
    ge.submap = h.submap_d;
  }
  h.nrep = nrep;
  if (h.big) {
    // HBM-resident Neumann records from the representative system's moduli
    double* emrep = Y + nsl * m;
    hipLaunchKernelGGL(k_moduli<double>, dim3(1024), dim3(kThreads), 0, st, rrep, emrep,
                       (int64_t)g.nel, pr.E0, pr.Emin, pr.penal);
    nin.g = g;
    nin.em = emrep;
    nin.fixed = h.fixed;
    nin.K0 = h.K0;
    nin.dis = dis;
    nin.shift = mp.shift;
    nin.fixed_diag = kFixedDiag;
    nin.neumann = 1;
    nin.nsys = 1;
    big_factor<double>(nin, nfac, fws, h.dflag, st);
  } else {
    StencilIn sn = si;
    sn.g = ge;
    sn.rho = rrep;
    sn.neumann = 1;
    sn.dis = dis;
    launch_factor<double>(nullptr, nfac, nrep, lsh, h.dflag, st, false, &sn);
  }
  hipLaunchKernelGGL(k_eig_init, dim3(nrep), dim3(kThreads), 0, st, ge, X, dis, m);
  hipLaunchKernelGGL(k_eig_cholqr, dim3(nrep), dim3(kThreads), 0, st, ge, X, dis, m);
  for (int it = 0; it < iters; ++it) {
    if (h.big) big_solve_multi(nin, nfac, m, X, Y, fws, st);
    else launch_solve_multi(nfac, lsh, nrep, m, X, Y, st);
    hipLaunchKernelGGL(k_eig_cholqr, dim3(nrep), dim3(kThreads), 0, st, ge, Y, dis, m);
    std::swap(X, Y);
  }
  if (g.dim == 2)
    hipLaunchKernelGGL(k_neumann_apply<2>, dim3(nrep), dim3(kThreads), 0, st, ge, rrep, h.K0, dis,
                       X, Y, m, mp);
  else
    hipLaunchKernelGGL(k_neumann_apply<3>, dim3(nrep), dim3(kThreads), 0, st, ge, rrep, h.K0, dis,
                       X, Y, m, mp);
  hipLaunchKernelGGL(k_eig_rr, dim3(nrep), dim3(kThreads), 0, st, ge, X, Y, dis, m, h.lam,
                     h.eres, h.phi, pr.lambda_thresh, h.kj);
  if (npairs > 0)
    hipLaunchKernelGGL(k_dedup_scatter, dim3(npairs), dim3(kThreads), 0, st, g, h.dedup_pairs,
                       h.phi, h.lam, h.eres, h.kj, m);
  if (h.mixed)
    hipLaunchKernelGGL(k_phi_modes<float>, dim3(1024), dim3(kThreads), 0, st, g, h.phi,
                       reinterpret_cast<float*>(h.phim));
  else
    hipLaunchKernelGGL(k_phi_modes<double>, dim3(1024), dim3(kThreads), 0, st, g, h.phi,
                       reinterpret_cast<double*>(h.phim));

  }

  // --- 4: coarse matrices and factors, all systems per launch ---
  double* W = h.build_ws;                 // [nsys][wsz]
  double* Ac = W + wsz * nsys;
  double* Sc = Ac + asm_coarse * nsys;    // dense coarse path: K_c's tiles, then the sweep's work
  const bool dense = g.nt <= g.dense_max && !g.cband;
  double* cws = Sc + (dense ? (size_t)nsys * big_nl(big_ntb(g.nt)) * kBTE : 0);
  double* bws = Sc + (dense ? coarse_dense_ws_elems(g, nsys)
                            : (g.cband ? coarse_band_ws_elems(g, nsys) : 0));   // big local factors
  hipMemsetAsync(Ac, 0, sizeof(double) * asm_coarse * nsys, st);
  const int nnb = g.dim == 3 ? 27 : 9;
  {
    const dim3 wgrid(g.nsub, nsys);
    if (g.dim == 2 && g.k <= 8)
      hipLaunchKernelGGL((k_coarse_W<2, 8>), wgrid, dim3(kThreads), 0, st, g, rho, h.K0, h.fixed,
                         h.phi, W, wsz, mp);
    else if (g.dim == 2)
      hipLaunchKernelGGL((k_coarse_W<2, kMaxK>), wgrid, dim3(kThreads), 0, st, g, rho, h.K0,
                         h.fixed, h.phi, W, wsz, mp);
    else if (g.k <= 8)
      hipLaunchKernelGGL((k_coarse_W<3, 8>), wgrid, dim3(kThreads), 0, st, g, rho, h.K0, h.fixed,
                         h.phi, W, wsz, mp);
    else
      hipLaunchKernelGGL((k_coarse_W<3, kMaxK>), wgrid, dim3(kThreads), 0, st, g, rho, h.K0,
                         h.fixed, h.phi, W, wsz, mp);
  }
  if (g.dim == 2)
    hipLaunchKernelGGL(k_coarse_assemble_mma<2>, dim3(g.nsub * nnb, nsys), dim3(kThreads), 0, st,
                       g, h.phi, W, wsz, Ac, asm_coarse, h.kj);
  else
    hipLaunchKernelGGL(k_coarse_assemble_mma<3>, dim3(g.nsub * nnb, nsys), dim3(kThreads), 0, st,
                       g, h.phi, W, wsz, Ac, asm_coarse, h.kj);
  hipEventRecord(h.fork, st);
  hipStreamWaitEvent(h.side, h.fork, 0);

  // --- 5 (second stream, beside the coarse factorisation, which occupies
  //     only one workgroup per system, and the coarse inverse): local
  //     Dirichlet factors as tiled C_b records (FP32 in mixed mode), all
  //     systems in one launch, and the moduli their layer couplings use ---
  {
    hipStream_t s2 = h.side;
    const size_t trec = (size_t)g.nsub * g.nblk * tile_shape(g.nb).tstride;
    const int64_t nm = (int64_t)nsys * g.nel;
    StencilIn sd = si;
    sd.neumann = 0;
    sd.dis = nullptr;
    sd.twist = h.twist;
    if (h.big) {
      double* em = h.mixed ? h.emod64 : reinterpret_cast<double*>(h.emod);
      hipLaunchKernelGGL(k_moduli<double>, dim3(1024), dim3(kThreads), 0, s2, rho, em, nm, pr.E0,
                         pr.Emin, pr.penal);
      BigFactorIn din{};
      din.g = g;
      din.em = em;
      din.fixed = h.fixed;
      din.K0 = h.K0;
      din.neumann = 0;
      din.nsys = nsys;
      if (h.mixed) big_factor<float>(din, reinterpret_cast<float*>(h.lfac), bws, h.dflag, s2);
      else big_factor<double>(din, reinterpret_cast<double*>(h.lfac), bws, h.dflag, s2);
    } else if (local_factor_fits(g)) {
      // FP64 moduli for the factorisations: those the solves use, or in
      // mixed precision a separate FP64 copy
      double* em = h.mixed ? h.emod64 : reinterpret_cast<double*>(h.emod);
      hipLaunchKernelGGL(k_moduli<double>, dim3(1024), dim3(kThreads), 0, s2, rho, em, nm, pr.E0,
                         pr.Emin, pr.penal);
      sd.emod = em;
      if (h.mixed)
        launch_local_factor<float>(sd, reinterpret_cast<float*>(h.lfac), h.dflag, nsys, trec, s2);
      else
        launch_local_factor<double>(sd, reinterpret_cast<double*>(h.lfac), h.dflag, nsys, trec,
                                    s2);
    } else {
      for (int sys = 0; sys < nsys; ++sys) {   // one system at a time (shared twist scratch)
        sd.rho = rho + (size_t)sys * g.nel;
        if (h.mixed)
          launch_factor<float>(nullptr, reinterpret_cast<float*>(h.lfac) + sys * trec, g.nsub,
                               lsh, h.dflag, s2, true, &sd);
        else
          launch_factor<double>(nullptr, reinterpret_cast<double*>(h.lfac) + sys * trec, g.nsub,
                                lsh, h.dflag, s2, true, &sd);
      }
      if (!h.mixed)
        hipLaunchKernelGGL(k_moduli<double>, dim3(1024), dim3(kThreads), 0, s2, rho,
                           reinterpret_cast<double*>(h.emod), nm, pr.E0, pr.Emin, pr.penal);
    }
    if (h.mixed)
      hipLaunchKernelGGL(k_moduli<float>, dim3(1024), dim3(kThreads), 0, s2, rho,
                         reinterpret_cast<float*>(h.emod), nm, pr.E0, pr.Emin, pr.penal);
    hipEventRecord(h.join, s2);
  }

  // coarse level: the dense K_c^-1 (its lower tiles feed the coarse
  // product), from the block-tridiagonal factor and its column-chunk inverse
  // when the coarse blocks fit those on-chip kernels, else by the block
  // sweep on the matrix cores; for coarse spaces too large for a dense
  // inverse, the block-tridiagonal factor alone
  if (g.cband) {
    coarse_band_factor(g, Ac, asm_coarse, nsys, h.cband, Sc, h.dflag, st);
  } else if (h.cpk && !coarse_btri_fits(g)) {
    coarse_dense_inverse(g, Ac, asm_coarse, nsys, Sc, cws, h.cpk, h.dflag, st);
  } else {
    launch_factor<double>(Ac, h.cfac, nsys, csh, h.dflag, st);
    if (h.cpk) {
      launch_inverse(h.cfac, csh, nsys, Sc, st);   // dense K_c^-1 in the coarse work area
      coarse_pack_inverse(g, Sc, nsys, h.cpk, st);
    }
  }

  hipStreamWaitEvent(st, h.join, 0);
  hipStreamSynchronize(st);

  int flag[4] = {0, 0, 0, 0};
  hipMemcpy(flag, h.dflag, sizeof(flag), hipMemcpyDeviceToHost);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    h.err = std::string("HIP error during setup: ") + hipGetErrorString(e);
    h.sticky = 1;
    return TPCG_EHIP;
  }
  if (flag[0]) {
    h.err = "non-positive pivot in a block Cholesky factorisation";
    return TPCG_ENOTSPD;
  }
  h.nsys_built = nsys;
  h.basis_ready = 1;
  return TPCG_OK;
}

}  // namespace tpcg
