// Two-level additive Schwarz preconditioner application (Sec. 2.4.2 with the
// additive form; coarse space of Sec. 2.4):
//   z = sum_j R_j^T A_j^-1 R_j r + Phi K_c^-1 Phi^T r
// in four launches:
//   1. restriction y_c = Phi^T r            (one or more workgroups per subdomain)
//   2. local solves A_j^-1 R_j r for every (system, subdomain)   } concurrent:
//   3. coarse solve x_c = K_c^-1 y_c                             } forked stream
//   4. extension z(n) = sum_{j owns n} (zloc_j(n) + (Phi_j x_c,j)(n)), with
//      the fused partial sums of r.z (and r.z_old for the flexible beta).
#include "big.h"
#include "btri.h"

namespace tpcg {

namespace {

constexpr int kSubThreads = 256;    // restriction: one workgroup per subdomain
constexpr int kXcStage = 2048;      // extension: coarse-solution entries staged per workgroup

// nsplit workgroups per subdomain (restrict_splits: more than one where a
// launch of one per subdomain would leave the chip unevenly loaded), all
// running systems together (Phi, mode-major, read once); KM >= k bounds the
// accumulators. Part s of box j takes the box DOFs [s nloc / nsplit,
// (s + 1) nloc / nsplit); with nsplit = 1 the sums go to y_c, else to ycp
// [nsplit][kMaxSys][nt], which k_restrict_sum adds up in part order.
template <typename P, int KM>
__global__ __launch_bounds__(kSubThreads) void k_restrict(Geometry g, const P* __restrict__ phim,
                                                          const double* __restrict__ r,
                                                          double* __restrict__ yc,
                                                          double* __restrict__ ycp,
                                                          const int* __restrict__ kj, int nsys,
                                                          int nsplit, Gate gate) {
  constexpr int NW = kSubThreads / 64;
  __shared__ double red[NW][kMaxSys * KM];
  // systems still running after the previous test (a superset of those that
  // pass this iteration's test, which is taken below, after the loads)
  unsigned run = 0;
  for (int sys = 0; sys < nsys; ++sys)
    if (gate_running(gate, sys)) run |= 1u << sys;
  if (!run) return;
  // XCD-aware order: the workgroups whose index agrees mod 8 share an XCD
  // and take a contiguous range of boxes, whose shared faces of r meet in
  // one L2
  const int W = gridDim.x, grp = blockIdx.x % 8, per = W / 8, rem = W % 8;
  const int slot = (grp < rem ? grp * (per + 1) : rem * (per + 1) + (grp - rem) * per) +
                   blockIdx.x / 8;
  const int j = slot / nsplit, part = slot - (slot / nsplit) * nsplit;
  const int lbeg = (int)((int64_t)part * g.nloc / nsplit);
  const int lend = (int)((int64_t)(part + 1) * g.nloc / nsplit);
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  const int k = g.k;
  // the box's vectors in use: the other columns of Phi_j are zero, their
  // entries of y_c stay zero
  const int ku = kj[j];
  const P* ph = phim + (size_t)j * k * g.nloc;
  double acc[kMaxSys][KM];
#pragma unroll
  for (int q = 0; q < kMaxSys; ++q)
#pragma unroll
    for (int m = 0; m < KM; ++m) acc[q][m] = 0.0;
  // kRU box DOFs per thread at a time, all their loads issued before use
  // (one with the wide accumulators, which fill the registers)
  constexpr int kRU = KM <= 8 ? 5 : 1;
  for (int l0 = lbeg + threadIdx.x; l0 < lend; l0 += kRU * kSubThreads) {
    double rv[kRU][kMaxSys];
#pragma unroll
    for (int u = 0; u < kRU; ++u) {
      const int l = l0 + u * kSubThreads;
      const int64_t dof = l < lend ? box_dof(g, jx, jy, jz, l) : 0;
#pragma unroll
      for (int q = 0; q < kMaxSys; ++q)
        rv[u][q] = (l < lend && ((run >> q) & 1u)) ? r[q * g.ndof + dof] : 0.0;
    }
    // modes in groups of eight, the group's loads issued together
#pragma unroll
    for (int m0 = 0; m0 < KM; m0 += 8)
      if (m0 < ku) {
        double pv[8][kRU];
        if constexpr (sizeof(P) == 4) {
          // FP32 copy: every load from a valid address (entry 0 of the box
          // when out of range) and no branch around it, all issued before the
          // first product; a load guarded by a branch was waited for inside
          // the branch, where its conversion sat, which serialised the group
          P raw[8][kRU];
#pragma unroll
          for (int mm = 0; mm < 8; ++mm)
#pragma unroll
            for (int u = 0; u < kRU; ++u) {
              const int l = l0 + u * kSubThreads, m = m0 + mm;
              raw[mm][u] = ph[(m < ku && l < lend) ? (size_t)m * g.nloc + l : 0];
            }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int mm = 0; mm < 8; ++mm)
#pragma unroll
            for (int u = 0; u < kRU; ++u) {
              const int l = l0 + u * kSubThreads, m = m0 + mm;
              pv[mm][u] = (m < ku && l < lend) ? (double)raw[mm][u] : 0.0;
            }
        } else {
#pragma unroll
          for (int mm = 0; mm < 8; ++mm)
#pragma unroll
            for (int u = 0; u < kRU; ++u) {
              const int l = l0 + u * kSubThreads, m = m0 + mm;
              pv[mm][u] = (m < ku && l < lend) ? (double)ph[(size_t)m * g.nloc + l] : 0.0;
            }
        }
#pragma unroll
        for (int mm = 0; mm < 8; ++mm)
#pragma unroll
          for (int u = 0; u < kRU; ++u)
#pragma unroll
            for (int q = 0; q < kMaxSys; ++q) acc[q][m0 + mm] += pv[mm][u] * rv[u][q];
      }
  }
  const int w = threadIdx.x >> 6;
  if (gate.test && gate.enabled) {
    // this iteration's residual test, all systems in one reduction (the same
    // order in every workgroup); workgroup 0 publishes the flags
    __shared__ double tst[NW][kMaxSys];
    double rr[kMaxSys];
#pragma unroll
    for (int q = 0; q < kMaxSys; ++q) rr[q] = 0.0;
    double* parts = const_cast<double*>(gate.parts);
    for (int i = threadIdx.x; i < gate.np; i += kSubThreads)
#pragma unroll
      for (int q = 0; q < kMaxSys; ++q)
        if ((run >> q) & 1u) rr[q] += part_slot(parts, gate.rr_slot, q)[i];
#pragma unroll
    for (int q = 0; q < kMaxSys; ++q) {
      const double v = wave_sum(rr[q]);
      if ((threadIdx.x & 63) == 0) tst[w][q] = v;
    }
    __syncthreads();
    int* istate = const_cast<int*>(gate.istate);
    for (int sys = 0; sys < nsys; ++sys) {
      if (!((run >> sys) & 1u)) continue;
      double v = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) v += tst[w2][sys];
      const bool go = v > gate.tol2 * scal_slot(parts, kScFF)[sys];
      if (!go) run &= ~(1u << sys);
      if (blockIdx.x == 0 && threadIdx.x == 0) istate[kStRun * kMaxSys + sys] = go ? 1 : 0;
    }
  }
#pragma unroll
  for (int q = 0; q < kMaxSys; ++q)
#pragma unroll
    for (int m = 0; m < KM; ++m)
      if (m < k && ((run >> q) & 1u)) {
        const double v = wave_sum(acc[q][m]);
        if ((threadIdx.x & 63) == 0) red[w][q * KM + m] = v;
      }
  __syncthreads();
  for (int i = threadIdx.x; i < nsys * k; i += kSubThreads) {
    const int q = i / k, m = i - (i / k) * k;
    if (!((run >> q) & 1u)) continue;
    const int e = q * KM + m;
    double s = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < NW; ++w2) s += red[w2][e];
    const int ci = coarse_index(g, jx, jy, jz, m);
    if (nsplit == 1) yc[(size_t)q * g.nt + ci] = s;
    else ycp[((size_t)part * kMaxSys + q) * g.nt + ci] = s;
  }
}

// y_c = the sum of the parts of k_restrict, in part order, for the systems
// that passed the residual test taken there. grid (ceil(nt / 256), nsys).
__global__ __launch_bounds__(kThreads) void k_restrict_sum(Geometry g,
                                                          const double* __restrict__ ycp,
                                                          double* __restrict__ yc, int nsplit,
                                                          Gate gate) {
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= g.nt) return;
  double s = 0.0;
  for (int p = 0; p < nsplit; ++p) s += ycp[((size_t)p * kMaxSys + sys) * g.nt + i];
  yc[(size_t)sys * g.nt + i] = s;
}

// one workgroup per system
template <int MAXV>
__global__ __launch_bounds__(kThreads) void k_coarse_solve(Geometry g, const double* __restrict__ cfac,
                                                          const double* __restrict__ yc,
                                                          double* __restrict__ xc, Gate gate) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int sys = blockIdx.x;
  if (!gate_running(gate, sys)) return;
  const BtriShape shp = coarse_shape(g);
  const double* fac = cfac + (size_t)sys * g.nblkc * g.bstridec;
  const double* ys = yc + (size_t)sys * g.nt;
  double* xs = xc + (size_t)sys * g.nt;
  const int nbc = g.nbc;
  btri_solve<double, 1, MAXV>(
      fac, shp, 1, [&](int b, int i, int) { return ys[b * nbc + i]; },
      [&](int b, int i, int) -> double& { return xs[b * nbc + i]; }, smem);
}

// Tile (I, J), I >= J, of the lower tiles in row-major tile order.
__device__ inline void coarse_tile_ij(int tile, int& I, int& J) {
  I = 0;
  while ((I + 1) * (I + 2) / 2 <= tile) ++I;
  J = tile - I * (I + 1) / 2;
}

// Partial products of x_c = K_c^-1 y_c from the packed lower tiles, for the
// running systems: tile (I, J) writes K_IJ y_J into slot [I][J] of row block
// I and, below the diagonal, K_IJ^T y_I into slot [J][I] of row block J, so
// every slot is written once. Wave w holds rows 16 w .. 16 w + 15 of the
// tile, lane l column l (each row read as 512 contiguous bytes). Row sums go
// through LDS (padded rows), column sums over the four waves.
// grid (T (T + 1) / 2, nsys).
__global__ __launch_bounds__(kThreads) void k_coarse_gemv_tiles(Geometry g,
                                                               const double* __restrict__ cpk,
                                                               const double* __restrict__ yc,
                                                               double* __restrict__ cpart,
                                                               Gate gate) {
  __shared__ double rows[4][16][kCT + 1];
  __shared__ double cols[4][kCT];
  const int sys = blockIdx.y, tile = blockIdx.x, nt = g.nt;
  if (!gate_running(gate, sys)) return;
  const int T = coarse_tiles(nt);
  int I, J;
  coarse_tile_ij(tile, I, J);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  const double* A = cpk + ((size_t)sys * (T * (T + 1) / 2) + tile) * kCT * kCT + 16 * w * kCT;
  const double* y = yc + (size_t)sys * nt;
  double a[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) a[q] = A[q * kCT + l];
  const int cj = J * kCT + l, ri = I * kCT + 16 * w;
  const double yj = cj < nt ? y[cj] : 0.0;
  double cs = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    rows[w][q][l] = a[q] * yj;
    cs += a[q] * (ri + q < nt ? y[ri + q] : 0.0);
  }
  cols[w][l] = cs;
  __syncthreads();
  double* P = cpart + (size_t)sys * T * T * kCT;
  {
    // lane l: row l / 4 of the wave's 16, columns 16 (l % 4) .. + 15
    const int q = l >> 2, h = l & 3;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += rows[w][q][16 * h + k];
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (h == 0) P[((size_t)I * T + J) * kCT + 16 * w + q] = s;
  }
  if (I != J && w == 0)
    P[((size_t)J * T + I) * kCT + l] = (cols[0][l] + cols[1][l]) + (cols[2][l] + cols[3][l]);
}

// x_c = the sum of a row block's T slots, in slot order. grid (ceil(nt /
// 256), nsys).
__global__ __launch_bounds__(kThreads) void k_coarse_gemv_sum(Geometry g,
                                                             const double* __restrict__ cpart,
                                                             double* __restrict__ xc, Gate gate) {
  const int sys = blockIdx.y, nt = g.nt;
  if (!gate_running(gate, sys)) return;
  const int r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= nt) return;
  const int T = coarse_tiles(nt);
  const double* P = cpart + ((size_t)sys * T * T + (size_t)(r / kCT) * T) * kCT + r % kCT;
  double s = 0.0;
  for (int K0 = 0; K0 < T; K0 += 16) {   // sixteen reads in flight, added in slot order
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = K0 + u < T ? P[(size_t)(K0 + u) * kCT] : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) s += v[u];
  }
  xc[(size_t)sys * nt + r] = s;
}

// z(n) = P sum_{j owns n} (zloc_j(n) + (Phi_j x_c,j)(n)) for every running
// system: the local solutions and the prolonged coarse solution in one pass
// (Phi mode-major, [nsub][k][nloc], read along box rows), with the fused
// partial sums of r.z (and r.z_old for the flexible beta).
template <typename T, int D, int KM>
__global__ __launch_bounds__(kThreads) void k_extend(
    Geometry g, const double* __restrict__ r, double* __restrict__ z, const T* __restrict__ zloc,
    const T* __restrict__ phim, const double* __restrict__ xc, const int* __restrict__ kj,
    const uint8_t* __restrict__ fixed, double* __restrict__ parts, int rz_slot, int flexible,
    int nsys, Gate gate) {
  __shared__ double sh[4];
  __shared__ double xs[kXcStage];
  unsigned run = 0;
  for (int sys = 0; sys < nsys; ++sys)
    if (gate_running(gate, sys)) run |= 1u << sys;
  if (!run) return;
  constexpr int d = D;
  const int s = g.s, k = g.k;
  const size_t zstride = (size_t)g.nsub * g.nloc;
  // XCD-aware order (workgroups whose index agrees mod 8 share an XCD): each
  // such group takes a contiguous range of node chunks, so the box rows that
  // neighbouring chunks both read meet in one L2
  const int W = gridDim.x, grp = blockIdx.x % 8, per = W / 8, rem = W % 8;
  const int slot = (grp < rem ? grp * (per + 1) : rem * (per + 1) + (grp - rem) * per) +
                   blockIdx.x / 8;
  double arz[kMaxSys], arzo[kMaxSys];
#pragma unroll
  for (int q = 0; q < kMaxSys; ++q) arz[q] = arzo[q] = 0.0;
  for (int64_t base = (int64_t)slot * kThreads; base < g.nnodes;
       base += (int64_t)gridDim.x * kThreads) {
    // x_c of the boxes this chunk of nodes can touch (every box column of
    // its node rows) staged in LDS; x_c from global memory when they do not fit
    const int64_t last = min(base + (int64_t)kThreads, g.nnodes) - 1;
    const int64_t r0 = base / g.nnx, r1 = last / g.nnx;   // node rows, iy + nny iz
    const int iy0 = (int)(r0 % g.nny), iz0 = (int)(r0 / g.nny);
    const int iy1 = (int)(r1 % g.nny), iz1 = (int)(r1 / g.nny);
    int ylo = iy0 == 0 ? 0 : (iy0 - 1) / s, yhi = min(g.gy - 1, iy1 / s);
    if (iz1 != iz0) { ylo = 0; yhi = g.gy - 1; }
    const int zlo = d == 3 ? (iz0 == 0 ? 0 : (iz0 - 1) / s) : 0;
    const int zhi = d == 3 ? min(g.gz - 1, iz1 / s) : 0;
    const int ny = yhi - ylo + 1;
    const int cnt = g.gx * ny * (zhi - zlo + 1) * k;
    const bool staged = cnt * nsys <= kXcStage;
    __syncthreads();   // the previous chunk's reads of xs are done
    if (staged)
      for (int e = threadIdx.x; e < cnt * nsys; e += kThreads) {
        const int q = e / cnt, rr = e - q * cnt;
        const int box = rr / k, m = rr - box * k;
        const int jx = box % g.gx, jy = ylo + (box / g.gx) % ny, jz = zlo + box / (g.gx * ny);
        xs[e] = ((run >> q) & 1u) ? xc[(size_t)q * g.nt + coarse_index(g, jx, jy, jz, m)] : 0.0;
      }
    __syncthreads();
    const int64_t n = base + threadIdx.x;
    if (n >= g.nnodes) continue;
    const int ix = (int)(n % g.nnx);
    const int iy = (int)((n / g.nnx) % g.nny);
    const int iz = (int)(n / ((int64_t)g.nnx * g.nny));
    const int x0 = ix == 0 ? 0 : (ix - 1) / s, x1 = min(g.gx - 1, ix / s);
    const int y0 = iy == 0 ? 0 : (iy - 1) / s, y1 = min(g.gy - 1, iy / s);
    int z0 = 0, z1 = 0;
    if (d == 3) { z0 = iz == 0 ? 0 : (iz - 1) / s; z1 = min(g.gz - 1, iz / s); }
    // a node lies in at most two subdomains along each axis (overlap of one
    // cell); per subdomain: its local solution, then the prolonged coarse
    // solution mode by mode
    double acc[kMaxSys][3];
#pragma unroll
    for (int q = 0; q < kMaxSys; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
#pragma unroll
    for (int cz = 0; cz < D - 1; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          const int jx = x0 + cx, jy = y0 + cy, jz = z0 + cz;
          if (jx > x1 || jy > y1 || jz > z1) continue;
          const int j = jx + g.gx * (jy + g.gy * jz);
          const int ln = (ix - s * jx) + g.bn * ((iy - s * jy) + g.bn * (iz - s * jz));
          const T* zj = zloc + (size_t)j * g.nloc + (size_t)d * ln;
          const T* pj = phim + (size_t)j * k * g.nloc + (size_t)d * ln;
          const double* xj = xc + coarse_index(g, jx, jy, jz, 0);
          const int sb = ((jz - zlo) * ny + (jy - ylo)) * g.gx + jx;   // staged box
          if constexpr (D == 2) {
            typedef T T2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int q = 0; q < kMaxSys; ++q)
              if ((run >> q) & 1u) {
                const T2 v = *reinterpret_cast<const T2*>(zj + q * zstride);
                acc[q][0] += (double)v.x;
                acc[q][1] += (double)v.y;
              }
          } else {
#pragma unroll
            for (int q = 0; q < kMaxSys; ++q)
              if ((run >> q) & 1u)
#pragma unroll
                for (int c = 0; c < D; ++c) acc[q][c] += (double)zj[q * zstride + c];
          }
          // modes in groups of eight: the group's basis values loaded together
          // (only the box's vectors in use: the other columns are zero)
          const int ku = kj[j];
#pragma unroll
          for (int m0 = 0; m0 < KM; m0 += 8) {
            if (m0 >= ku) break;
            double pv[8][D];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int m = m0 + u;
              if constexpr (D == 2) {
                typedef T T2 __attribute__((ext_vector_type(2)));
                const T2 v = m < ku ? *reinterpret_cast<const T2*>(pj + (size_t)m * g.nloc) : T2{0, 0};
                pv[u][0] = (double)v.x;
                pv[u][1] = (double)v.y;
              } else if constexpr (sizeof(T) == 4) {
                // FP32 copy: loads from a valid address without a branch (as
                // in the restriction), then the conversion
                T raw[D];
#pragma unroll
                for (int c = 0; c < D; ++c) raw[c] = pj[m < ku ? (size_t)m * g.nloc + c : 0];
#pragma unroll
                for (int c = 0; c < D; ++c) pv[u][c] = m < ku ? (double)raw[c] : 0.0;
              } else {
#pragma unroll
                for (int c = 0; c < D; ++c) pv[u][c] = m < ku ? (double)pj[(size_t)m * g.nloc + c] : 0.0;
              }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int m = m0 + u;
              if (m < ku) {
#pragma unroll
                for (int q = 0; q < kMaxSys; ++q)
                  if ((run >> q) & 1u) {
                    const double xv =
                        staged ? xs[(q * cnt / k + sb) * k + m] : xj[(size_t)q * g.nt + m];
#pragma unroll
                    for (int c = 0; c < D; ++c) acc[q][c] += pv[u][c] * xv;
                  }
              }
            }
          }
        }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const int64_t i = d * n + c;
      const bool f = fixed[i];
#pragma unroll
      for (int q = 0; q < kMaxSys; ++q) {
        if (!((run >> q) & 1u)) continue;
        const double zn = f ? 0.0 : acc[q][c];
        const double ri = r[q * g.ndof + i];
        double* zq = z + q * g.ndof;
        if (flexible) arzo[q] += ri * zq[i];
        zq[i] = zn;
        arz[q] += ri * zn;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kMaxSys; ++q) {
    if (!((run >> q) & 1u)) continue;
    const double v = block_sum(arz[q], sh);
    if (threadIdx.x == 0) part_slot(parts, rz_slot, q)[slot] = v;
    if (flexible) {
      const double w = block_sum(arzo[q], sh);
      if (threadIdx.x == 0) part_slot(parts, kPartRZO, q)[slot] = w;
    }
  }
}

template <typename K>
void set_lds_once(K kernel, bool& done) {
  if (done) return;
  hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();   // an unsupported size must not leave a stale error behind
  done = true;
}

#define TPCG_COARSE_CASE(V)                                                                 \
  case V: {                                                                                 \
    static bool done = false;                                                               \
    set_lds_once(&k_coarse_solve<V>, done);                                                 \
    hipLaunchKernelGGL(k_coarse_solve<V>, dim3(nsys), dim3(kThreads), lds, st, g, h.cfac,   \
                       h.yc, h.xc, gate);                                                   \
    break;                                                                                  \
  }

void coarse_launch(Handle& h, int nsys, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  const size_t lds = sizeof(double) * btri_solve_lds_elems(coarse_shape(g), 1);
  switch (stage_bucket(stage_regs_for<double>(g.nbc, g.pec))) {
    TPCG_COARSE_CASE(2)
    TPCG_COARSE_CASE(5)
    TPCG_COARSE_CASE(10)
    TPCG_COARSE_CASE(16)
    TPCG_COARSE_CASE(24)
    TPCG_COARSE_CASE(36)
    default: break;
  }
}

// Phi^T r for every running system (T: precision of the iteration copy of Phi)
template <typename T>
void restrict_launch(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  const T* pm = reinterpret_cast<const T*>(h.phim);
  const int ns = restrict_splits(g);
  const dim3 grid(g.nsub * ns);
  if (g.k <= 8)
    hipLaunchKernelGGL((k_restrict<T, 8>), grid, dim3(kSubThreads), 0, st, g, pm, r, h.yc, h.ycp,
                       h.kj, nsys, ns, gate);
  else
    hipLaunchKernelGGL((k_restrict<T, kMaxK>), grid, dim3(kSubThreads), 0, st, g, pm, r, h.yc,
                       h.ycp, h.kj, nsys, ns, gate);
  if (ns > 1) {
    Gate gs = gate;
    gs.test = 0;   // the test was taken in the restriction
    hipLaunchKernelGGL(k_restrict_sum, dim3((g.nt + kThreads - 1) / kThreads, nsys),
                       dim3(kThreads), 0, st, g, h.ycp, h.yc, ns, gs);
  }
}

// z = P sum_j R_j^T (zloc_j + Phi_j x_c,j) with the r.z partials
template <typename T>
void extend_launch(Handle& h, const double* r, double* z, int nsys, const Gate& gate, int rz_slot,
                   int flexible, hipStream_t st) {
  const Geometry& g = h.g;
  const T* pm = reinterpret_cast<const T*>(h.phim);
  const T* zl = reinterpret_cast<const T*>(h.zloc);
  const dim3 grid(parts_for(g.nnodes));
#define TPCG_EXTEND(D, KM)                                                                     \
  hipLaunchKernelGGL((k_extend<T, D, KM>), grid, dim3(kThreads), 0, st, g, r, z, zl, pm, h.xc,  \
                     h.kj, h.fixed, h.parts, rz_slot, flexible, nsys, gate)
  if (g.dim == 2) {
    if (g.k <= 8) TPCG_EXTEND(2, 8);
    else TPCG_EXTEND(2, kMaxK);
  } else {
    if (g.k <= 8) TPCG_EXTEND(3, 8);
    else TPCG_EXTEND(3, kMaxK);
  }
#undef TPCG_EXTEND
}

}  // namespace

int restrict_splits(const Geometry& g) {
  // about four workgroups per CU of 256, each part at least 2048 box DOFs
  int s = (4 * 256 + g.nsub - 1) / g.nsub;
  s = std::min(s, std::min(8, g.nloc / 2048));
  return std::max(s, 1);
}

void launch_precond(Handle& h, const double* r, double* z, int nsys, const Gate& gate,
                    int rz_slot, int prof_it, int flexible, hipStream_t st) {
  const Geometry& g = h.g;
  const bool cap = h.cap_ev != nullptr;   // inside a graph capture: its own event pairs
  const bool prof = !cap && h.prof_on && prof_it >= -1;
  if (prof && (size_t)(2 * h.prof_n + 2) > h.prof_ev.size()) {
    const size_t old = h.prof_ev.size();
    h.prof_ev.resize(old + 512, nullptr);
    h.prof_it.resize(h.prof_ev.size() / 2, 0);
    for (size_t i = old; i < h.prof_ev.size(); ++i) hipEventCreate(&h.prof_ev[i]);
  }
  auto mark = [&](int which) {
    if (prof) hipEventRecord(h.prof_ev[2 * h.prof_n + which], st);
    if (cap && prof_it >= 0) hipEventRecord(h.cap_ev[2 * h.cap_n + which], st);
  };
  if (h.mixed) restrict_launch<float>(h, r, nsys, gate, st);
  else restrict_launch<double>(h, r, nsys, gate, st);
  // The dense coarse product runs on the main stream ahead of the local
  // solves: both are HBM-bound, and side by side they slowed each other more
  // than the shorter one takes alone. The block-tridiagonal coarse solve (for
  // coarse spaces too large for a dense inverse) occupies one workgroup per
  // system and is latency-bound: it runs beside the local solves on the side
  // stream.
  const bool beside = h.cpk == nullptr;
  if (!beside) {
    const int T = coarse_tiles(g.nt);
    hipLaunchKernelGGL(k_coarse_gemv_tiles, dim3(T * (T + 1) / 2, nsys), dim3(kThreads), 0, st, g,
                       h.cpk, h.yc, h.cpart, gate);
    hipLaunchKernelGGL(k_coarse_gemv_sum, dim3((g.nt + kThreads - 1) / kThreads, nsys),
                       dim3(kThreads), 0, st, g, h.cpart, h.xc, gate);
  } else {
    hipEventRecord(h.fork, st);
    hipStreamWaitEvent(h.side, h.fork, 0);
    if (g.cband) coarse_band_solve(g, h.cband, h.yc, h.xc, h.cband_w, nsys, gate, h.side);
    else coarse_launch(h, nsys, gate, h.side);
    hipEventRecord(h.join, h.side);
  }
  mark(0);
  launch_local_solves(h, r, nsys, gate, st);
  mark(1);
  if (beside) hipStreamWaitEvent(st, h.join, 0);
  if (h.mixed) extend_launch<float>(h, r, z, nsys, gate, rz_slot, flexible, st);
  else extend_launch<double>(h, r, z, nsys, gate, rz_slot, flexible, st);
  if (prof) h.prof_it[h.prof_n++] = prof_it;
  if (cap && prof_it >= 0) ++h.cap_n;
}

void launch_coarse_only(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  if (h.mixed) restrict_launch<float>(h, r, nsys, gate, st);
  else restrict_launch<double>(h, r, nsys, gate, st);
  if (h.cpk) {
    const int T = coarse_tiles(g.nt);
    hipLaunchKernelGGL(k_coarse_gemv_tiles, dim3(T * (T + 1) / 2, nsys), dim3(kThreads), 0, st, g,
                       h.cpk, h.yc, h.cpart, gate);
    hipLaunchKernelGGL(k_coarse_gemv_sum, dim3((g.nt + kThreads - 1) / kThreads, nsys),
                       dim3(kThreads), 0, st, g, h.cpart, h.xc, gate);
  } else if (g.cband) {
    coarse_band_solve(g, h.cband, h.yc, h.xc, h.cband_w, nsys, gate, st);
  } else {
    coarse_launch(h, nsys, gate, st);
  }
}

}  // namespace tpcg
