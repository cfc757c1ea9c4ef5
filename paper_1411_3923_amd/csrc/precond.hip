// Two-level additive Schwarz preconditioner application (Sec. 2.4.2 with the
// additive form; coarse space of Sec. 2.4):
//   z = sum_j R_j^T A_j^-1 R_j r + Phi K_c^-1 Phi^T r
// in four launches:
//   1. restriction y_c = Phi^T r            (one workgroup per subdomain)
//   2. local solves A_j^-1 R_j r for every (system, subdomain)   } concurrent:
//   3. coarse solves K_c^-1 y_c, one workgroup per system        } forked stream
//   4. extension z(n) = sum_{j owns n} (A_j^-1 R_j r)(n) + Phi(n) x_c, with the
//      fused partial sums of r.z (and r.z_old for the flexible beta).
#include "btri.h"

namespace tpcg {

namespace {

// global DOF of local DOF l of subdomain (jx, jy, jz)
__device__ inline int64_t box_dof(const Geometry& g, int jx, int jy, int jz, int l) {
  const int d = g.dim;
  const int ln = l / d, c = l - ln * d;
  const int lx = ln % g.bn;
  const int rest = ln / g.bn;
  const int ly = rest % g.bn;
  const int lz = rest / g.bn;
  const int64_t n = (int64_t)(g.s * jx + lx) +
                    (int64_t)g.nnx * ((g.s * jy + ly) + (int64_t)g.nny * (g.s * jz + lz));
  return d * n + c;
}

__device__ inline void sub_coords(const Geometry& g, int j, int& jx, int& jy, int& jz) {
  jx = j % g.gx;
  jy = (j / g.gx) % g.gy;
  jz = j / (g.gx * g.gy);
}

template <typename P>
__global__ __launch_bounds__(kThreads) void k_restrict(Geometry g, const P* __restrict__ phi,
                                                       const double* __restrict__ r,
                                                       double* __restrict__ yc, int nsys,
                                                       Gate gate) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  const int k = g.k;
  const P* ph = phi + (size_t)j * g.nloc * k;
  for (int sys = 0; sys < nsys; ++sys) {
    if (!gate_running(gate, sys, sh)) continue;
    const double* rs = r + (size_t)sys * g.ndof;
    double acc[kMaxK];
#pragma unroll
    for (int m = 0; m < kMaxK; ++m) acc[m] = 0.0;
    for (int l = threadIdx.x; l < g.nloc; l += kThreads) {
      const double rv = rs[box_dof(g, jx, jy, jz, l)];
#pragma unroll
      for (int m = 0; m < kMaxK; ++m)
        if (m < k) acc[m] += (double)ph[(size_t)l * k + m] * rv;
    }
    for (int m = 0; m < k; ++m) {
      const double v = block_sum(acc[m], sh);
      if (threadIdx.x == 0) yc[(size_t)sys * g.nt + coarse_index(g, jx, jy, jz, m)] = v;
    }
  }
}

// one workgroup per (system, subdomain); factors and results in T
template <typename T, int MAXV>
__global__ __launch_bounds__(kThreads) void k_local_solves(Geometry g, const double* __restrict__ r,
                                                          const T* __restrict__ lfac,
                                                          T* __restrict__ zloc, Gate gate) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sh[4];
  const int sys = blockIdx.x / g.nsub;
  const int j = blockIdx.x - sys * g.nsub;
  if (!gate_running(gate, sys, sh)) return;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  const BtriShape shp = local_shape(g);
  const T* fac = lfac + ((size_t)sys * g.nsub + j) * g.nblk * g.bstride;
  const double* rs = r + (size_t)sys * g.ndof;
  T* zs = zloc + ((size_t)sys * g.nsub + j) * g.nloc;
  const int nb = g.nb;
  btri_solve<T, 1, MAXV>(
      fac, shp, 1, [&](int b, int i, int) { return rs[box_dof(g, jx, jy, jz, b * nb + i)]; },
      [&](int b, int i, int) -> T& { return zs[b * nb + i]; }, smem);
}

// one workgroup per system
template <int MAXV>
__global__ __launch_bounds__(kThreads) void k_coarse_solve(Geometry g, const double* __restrict__ cfac,
                                                          const double* __restrict__ yc,
                                                          double* __restrict__ xc, Gate gate) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sh[4];
  const int sys = blockIdx.x;
  if (!gate_running(gate, sys, sh)) return;
  const BtriShape shp = coarse_shape(g);
  const double* fac = cfac + (size_t)sys * g.nblkc * g.bstridec;
  const double* ys = yc + (size_t)sys * g.nt;
  double* xs = xc + (size_t)sys * g.nt;
  const int nbc = g.nbc;
  btri_solve<double, 1, MAXV>(
      fac, shp, 1, [&](int b, int i, int) { return ys[b * nbc + i]; },
      [&](int b, int i, int) -> double& { return xs[b * nbc + i]; }, smem);
}

// x_c = K_c^-1 y_c with the dense inverse: one wave per row, four rows per
// workgroup; grid.x = nsys * ceil(nt / 4)
__global__ __launch_bounds__(kThreads) void k_coarse_gemv(Geometry g, const double* __restrict__ cinv,
                                                         const double* __restrict__ yc,
                                                         double* __restrict__ xc, Gate gate) {
  __shared__ double sh[4];
  const int per_sys = (g.nt + 3) / 4;
  const int sys = blockIdx.x / per_sys;
  if (!gate_running(gate, sys, sh)) return;
  const int row = (blockIdx.x - sys * per_sys) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= g.nt) return;
  const double* a = cinv + ((size_t)sys * g.nt + row) * g.nt;
  const double* y = yc + (size_t)sys * g.nt;
  double s = 0.0;
  for (int c = lane; c < g.nt; c += 64) s += a[c] * y[c];
  s = wave_sum(s);
  if (lane == 0) xc[(size_t)sys * g.nt + row] = s;
}

template <typename T, typename P>
__global__ __launch_bounds__(kThreads) void k_extend(
    Geometry g, const double* __restrict__ r, double* __restrict__ z, const T* __restrict__ zloc,
    const P* __restrict__ phi, const double* __restrict__ xc, const uint8_t* __restrict__ fixed,
    double* __restrict__ parts, int rz_slot, int flexible, Gate gate) {
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys, sh)) return;
  const int d = g.dim, s = g.s, k = g.k;
  const double* rs = r + (size_t)sys * g.ndof;
  double* zs = z + (size_t)sys * g.ndof;
  const T* zl = zloc + (size_t)sys * g.nsub * g.nloc;
  const double* xs = xc + (size_t)sys * g.nt;
  double arz = 0.0, arzo = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < g.nnodes;
       n += (int64_t)gridDim.x * kThreads) {
    const int ix = (int)(n % g.nnx);
    const int iy = (int)((n / g.nnx) % g.nny);
    const int iz = (int)(n / ((int64_t)g.nnx * g.nny));
    const int x0 = ix == 0 ? 0 : (ix - 1) / s, x1 = min(g.gx - 1, ix / s);
    const int y0 = iy == 0 ? 0 : (iy - 1) / s, y1 = min(g.gy - 1, iy / s);
    int z0 = 0, z1 = 0;
    if (d == 3) { z0 = iz == 0 ? 0 : (iz - 1) / s; z1 = min(g.gz - 1, iz / s); }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int jz = z0; jz <= z1; ++jz)
      for (int jy = y0; jy <= y1; ++jy)
        for (int jx = x0; jx <= x1; ++jx) {
          const int j = jx + g.gx * (jy + g.gy * jz);
          const int ln = (ix - s * jx) + g.bn * ((iy - s * jy) + g.bn * (iz - s * jz));
          const T* zj = zl + (size_t)j * g.nloc + (size_t)d * ln;
          const P* pj = phi + ((size_t)j * g.nloc + (size_t)d * ln) * k;
          const double* xj = xs + coarse_index(g, jx, jy, jz, 0);
          for (int c = 0; c < d; ++c) {
            double v = (double)zj[c];
            for (int m = 0; m < k; ++m) v += (double)pj[c * k + m] * xj[m];
            acc[c] += v;
          }
        }
    for (int c = 0; c < d; ++c) {
      const int64_t i = d * n + c;
      const double zn = fixed[i] ? 0.0 : acc[c];
      const double ri = rs[i];
      if (flexible) arzo += ri * zs[i];
      zs[i] = zn;
      arz += ri * zn;
    }
  }
  const double v = block_sum(arz, sh);
  if (threadIdx.x == 0) part_slot(parts, rz_slot, sys)[blockIdx.x] = v;
  if (flexible) {
    const double w = block_sum(arzo, sh);
    if (threadIdx.x == 0) part_slot(parts, kPartRZO, sys)[blockIdx.x] = w;
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

#define TPCG_LOCAL_CASE(V)                                                                  \
  case V: {                                                                                 \
    static bool done = false;                                                               \
    set_lds_once(&k_local_solves<T, V>, done);                                              \
    hipLaunchKernelGGL((k_local_solves<T, V>), dim3(nsys * g.nsub), dim3(kThreads), lds, st, \
                       g, r, reinterpret_cast<const T*>(h.lfac), reinterpret_cast<T*>(h.zloc), \
                       gate);                                                               \
    break;                                                                                  \
  }

template <typename T>
void local_launch(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  const size_t lds = sizeof(T) * btri_solve_lds_elems(local_shape(g), 1);
  switch (stage_bucket(stage_regs_for<T>(g.nb, g.pe))) {
    TPCG_LOCAL_CASE(2)
    TPCG_LOCAL_CASE(5)
    TPCG_LOCAL_CASE(10)
    TPCG_LOCAL_CASE(16)
    TPCG_LOCAL_CASE(24)
    TPCG_LOCAL_CASE(36)
    default: break;
  }
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

}  // namespace

void launch_precond(Handle& h, const double* r, double* z, int nsys, const Gate& gate,
                    int rz_slot, int prof_it, int flexible, hipStream_t st) {
  const Geometry& g = h.g;
  const bool prof = h.prof_on && prof_it >= -1;
  if (prof && (size_t)(2 * h.prof_n + 2) > h.prof_ev.size()) {
    const size_t old = h.prof_ev.size();
    h.prof_ev.resize(old + 512, nullptr);
    h.prof_it.resize(h.prof_ev.size() / 2, 0);
    for (size_t i = old; i < h.prof_ev.size(); ++i) hipEventCreate(&h.prof_ev[i]);
  }
  auto mark = [&](int which) {
    if (prof) hipEventRecord(h.prof_ev[2 * h.prof_n + which], st);
  };
  dim3 egrid(parts_for(g.nnodes), nsys);
  if (h.mixed)
    hipLaunchKernelGGL(k_restrict<float>, dim3(g.nsub), dim3(kThreads), 0, st, g, h.phi32, r,
                       h.yc, nsys, gate);
  else
    hipLaunchKernelGGL(k_restrict<double>, dim3(g.nsub), dim3(kThreads), 0, st, g, h.phi, r,
                       h.yc, nsys, gate);
  // the coarse solves run beside the local ones on the side stream
  hipEventRecord(h.fork, st);
  hipStreamWaitEvent(h.side, h.fork, 0);
  if (h.cinv)
    hipLaunchKernelGGL(k_coarse_gemv, dim3(nsys * ((g.nt + 3) / 4)), dim3(kThreads), 0, h.side, g,
                       h.cinv, h.yc, h.xc, gate);
  else
    coarse_launch(h, nsys, gate, h.side);
  hipEventRecord(h.join, h.side);
  mark(0);
  if (h.mixed) local_launch<float>(h, r, nsys, gate, st);
  else local_launch<double>(h, r, nsys, gate, st);
  mark(1);
  hipStreamWaitEvent(st, h.join, 0);
  if (h.mixed)
    hipLaunchKernelGGL((k_extend<float, float>), egrid, dim3(kThreads), 0, st, g, r, z,
                       reinterpret_cast<const float*>(h.zloc), h.phi32, h.xc, h.fixed, h.parts,
                       rz_slot, flexible, gate);
  else
    hipLaunchKernelGGL((k_extend<double, double>), egrid, dim3(kThreads), 0, st, g, r, z,
                       reinterpret_cast<const double*>(h.zloc), h.phi, h.xc, h.fixed, h.parts,
                       rz_slot, flexible, gate);
  if (prof) h.prof_it[h.prof_n++] = prof_it;
}

}  // namespace tpcg
