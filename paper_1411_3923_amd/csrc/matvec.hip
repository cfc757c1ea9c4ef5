// Matrix-free stiffness product y = P K(rho) P x (Sec. 2.1 discrete system,
// Sec. 2.2 element stiffness K_e = (E_min + (E0 - E_min) rho_e^p) K0).
//
// One thread per node gathers the contributions of the node's elements: for
// each element e around the node, the rows of E_e K0 that belong to the node
// times the element's nodal displacements. No atomics; each output is written
// once. K0 lives in LDS; the SIMP modulus is evaluated in the kernel.
#include "tpcg_internal.h"

namespace tpcg {

namespace {

__global__ __launch_bounds__(kThreads) void k_apply_q4(
    Geometry g, const double* __restrict__ rho, const double* __restrict__ x,
    double* __restrict__ y, const uint8_t* __restrict__ fixed, const double* __restrict__ K0,
    double E0, double Emin, double penal, double* __restrict__ parts, Gate gate) {
  __shared__ double K0s[64];
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  if (threadIdx.x < 64) K0s[threadIdx.x] = K0[threadIdx.x];
  __syncthreads();
  const double* xs = x + (size_t)sys * g.ndof;
  double* ys = y + (size_t)sys * g.ndof;
  const double* rs = rho + (size_t)sys * g.nel;
  const int nnx = g.nnx;
  double acc = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < g.nnodes;
       n += (int64_t)gridDim.x * kThreads) {
    const int ix = (int)(n % nnx), iy = (int)(n / nnx);
    double y0 = 0.0, y1 = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      // the node is corner a of element (ex, ey); corners counter-clockwise
      const int ex = ix - ((a == 1) || (a == 2));
      const int ey = iy - (a >= 2);
      if (ex < 0 || ex >= g.nelx || ey < 0 || ey >= g.nely) continue;
      const double E = simp_modulus(rs[ex + (int64_t)g.nelx * ey], E0, Emin, penal);
      const int64_t n0 = ex + (int64_t)nnx * ey;
      const int64_t nd[4] = {n0, n0 + 1, n0 + 1 + nnx, n0 + nnx};
      double t0 = 0.0, t1 = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double2 u = *reinterpret_cast<const double2*>(xs + 2 * nd[b]);
        const double u0 = fixed[2 * nd[b]] ? 0.0 : u.x;
        const double u1 = fixed[2 * nd[b] + 1] ? 0.0 : u.y;
        t0 += K0s[(2 * a) * 8 + 2 * b] * u0 + K0s[(2 * a) * 8 + 2 * b + 1] * u1;
        t1 += K0s[(2 * a + 1) * 8 + 2 * b] * u0 + K0s[(2 * a + 1) * 8 + 2 * b + 1] * u1;
      }
      y0 += E * t0;
      y1 += E * t1;
    }
    const bool f0 = fixed[2 * n], f1 = fixed[2 * n + 1];
    if (f0) y0 = 0.0;
    if (f1) y1 = 0.0;
    *reinterpret_cast<double2*>(ys + 2 * n) = make_double2(y0, y1);
    if (parts) {
      const double2 xv = *reinterpret_cast<const double2*>(xs + 2 * n);
      acc += (f0 ? 0.0 : xv.x) * y0 + (f1 ? 0.0 : xv.y) * y1;
    }
  }
  if (parts) {
    const double v = block_sum(acc, sh);
    if (threadIdx.x == 0) parts[(size_t)sys * kMaxParts + blockIdx.x] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_apply_h8(
    Geometry g, const double* __restrict__ rho, const double* __restrict__ x,
    double* __restrict__ y, const uint8_t* __restrict__ fixed, const double* __restrict__ K0,
    double E0, double Emin, double penal, double* __restrict__ parts, Gate gate) {
  __shared__ double K0s[576];
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  for (int i = threadIdx.x; i < 576; i += kThreads) K0s[i] = K0[i];
  __syncthreads();
  const double* xs = x + (size_t)sys * g.ndof;
  double* ys = y + (size_t)sys * g.ndof;
  const double* rs = rho + (size_t)sys * g.nel;
  const int nnx = g.nnx, nny = g.nny;
  const int64_t lay = (int64_t)nnx * nny;
  double acc = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < g.nnodes;
       n += (int64_t)gridDim.x * kThreads) {
    const int ix = (int)(n % nnx);
    const int iy = (int)((n / nnx) % nny);
    const int iz = (int)(n / lay);
    double yv[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 8; ++a) {
      const int dx = (a & 3) == 1 || (a & 3) == 2;
      const int dy = (a & 3) >= 2;
      const int dz = a >= 4;
      const int ex = ix - dx, ey = iy - dy, ez = iz - dz;
      if (ex < 0 || ex >= g.nelx || ey < 0 || ey >= g.nely || ez < 0 || ez >= g.nelz) continue;
      const double E = simp_modulus(rs[ex + (int64_t)g.nelx * (ey + (int64_t)g.nely * ez)],
                                    E0, Emin, penal);
      const int64_t n0 = ex + nnx * (ey + (int64_t)nny * ez);
      const int64_t nd[8] = {n0, n0 + 1, n0 + 1 + nnx, n0 + nnx,
                             n0 + lay, n0 + lay + 1, n0 + lay + 1 + nnx, n0 + lay + nnx};
      double t[3] = {0.0, 0.0, 0.0};
      for (int b = 0; b < 8; ++b) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int64_t dof = 3 * nd[b] + c;
          const double u = fixed[dof] ? 0.0 : xs[dof];
#pragma unroll
          for (int i = 0; i < 3; ++i) t[i] += K0s[(3 * a + i) * 24 + 3 * b + c] * u;
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) yv[i] += E * t[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int64_t dof = 3 * n + i;
      const bool fx = fixed[dof];
      if (fx) yv[i] = 0.0;
      ys[dof] = yv[i];
      if (parts) acc += (fx ? 0.0 : xs[dof]) * yv[i];
    }
  }
  if (parts) {
    const double v = block_sum(acc, sh);
    if (threadIdx.x == 0) parts[(size_t)sys * kMaxParts + blockIdx.x] = v;
  }
}

}  // namespace

void launch_apply_K(const Handle& h, const double* rho, const double* x, double* y, int nsys,
                    int dot_slot, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  dim3 grid(parts_for(g.nnodes), nsys);
  double* parts = dot_slot >= 0 ? part_slot(h.parts, dot_slot, 0) : nullptr;
  const tpcg_problem& pr = h.prob;
  if (g.dim == 2)
    hipLaunchKernelGGL(k_apply_q4, grid, dim3(kThreads), 0, st, g, rho, x, y, h.fixed, h.K0,
                       pr.E0, pr.Emin, pr.penal, parts, gate);
  else
    hipLaunchKernelGGL(k_apply_h8, grid, dim3(kThreads), 0, st, g, rho, x, y, h.fixed, h.K0,
                       pr.E0, pr.Emin, pr.penal, parts, gate);
}

}  // namespace tpcg
