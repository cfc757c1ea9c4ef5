// Density pipeline and compliance sensitivities.
//   filter:      rho_tilde_e = sum_i w_ei rho_i / sum_i w_ei,
//                w_ei = max(0, rmin - |x_e - x_i|) over element centres
//                (Sec. 4.3; truncated at the mesh boundary)
//   projection:  rho_bar = [tanh(b eta) + tanh(b (rho_tilde - eta))] /
//                          [tanh(b eta) + tanh(b (1 - eta))]   (Sec. 4.3)
//   chain rule:  dc/drho_i = sum_e dc/drho_bar_e H'(rho_tilde_e) w_ei / sum_k w_ek
//   compliance:  c = f^T u; dc/drho_bar_e = -p (E0 - E_min) rho_e^(p-1) u_e^T K0 u_e
//                (Sec. 2.2 objective, Sec. 4.2)
#include "tpcg_internal.h"

namespace tpcg {

namespace {

struct Etas {
  double v[kMaxSys];
};

__device__ inline void elem_coords(const Geometry& g, int64_t e, int& ex, int& ey, int& ez) {
  ex = (int)(e % g.nelx);
  ey = (int)((e / g.nelx) % g.nely);
  ez = (int)(e / ((int64_t)g.nelx * g.nely));
}

// sum of the hat weights around element (ex, ey, ez) inside the mesh
__device__ inline double weight_sum(const Geometry& g, int ex, int ey, int ez, double rmin, int R) {
  double s = 0.0;
  const int R3 = g.dim == 3 ? R : 0;
  for (int dz = -R3; dz <= R3; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int x = ex + dx, y = ey + dy, z = ez + dz;
        if (x < 0 || x >= g.nelx || y < 0 || y >= g.nely || z < 0 || z >= g.nelz) continue;
        const double w = rmin - sqrt((double)(dx * dx + dy * dy + dz * dz));
        if (w > 0.0) s += w;
      }
  return s;
}

__device__ inline double heaviside(double x, double beta, double eta) {
  return (tanh(beta * eta) + tanh(beta * (x - eta))) / (tanh(beta * eta) + tanh(beta * (1.0 - eta)));
}

__device__ inline double heaviside_d(double x, double beta, double eta) {
  const double t = tanh(beta * (x - eta));
  return beta * (1.0 - t * t) / (tanh(beta * eta) + tanh(beta * (1.0 - eta)));
}

__global__ __launch_bounds__(kThreads) void k_filter_project(Geometry g, const double* __restrict__ rho,
                                                            double rmin, double beta, Etas eta,
                                                            int nsys, double* __restrict__ rt,
                                                            double* __restrict__ rb) {
  const int R = rmin > 1.0 ? (int)ceil(rmin) - 1 : 0;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < g.nel;
       e += (int64_t)gridDim.x * kThreads) {
    double v;
    if (R == 0) {
      v = rho[e];
    } else {
      int ex, ey, ez;
      elem_coords(g, e, ex, ey, ez);
      double num = 0.0, den = 0.0;
      const int R3 = g.dim == 3 ? R : 0;
      for (int dz = -R3; dz <= R3; ++dz)
        for (int dy = -R; dy <= R; ++dy)
          for (int dx = -R; dx <= R; ++dx) {
            const int x = ex + dx, y = ey + dy, z = ez + dz;
            if (x < 0 || x >= g.nelx || y < 0 || y >= g.nely || z < 0 || z >= g.nelz) continue;
            const double w = rmin - sqrt((double)(dx * dx + dy * dy + dz * dz));
            if (w <= 0.0) continue;
            num += w * rho[x + (int64_t)g.nelx * (y + (int64_t)g.nely * z)];
            den += w;
          }
      v = num / den;
    }
    rt[e] = v;
    for (int s = 0; s < nsys; ++s) rb[(size_t)s * g.nel + e] = heaviside(v, beta, eta.v[s]);
  }
}

// ge[s][e] = gin[s][e] H'(rt_e) / sum_k w_ek: the adjoint's factor of each
// element (the weight sum and the projection's derivative once per element)
__global__ __launch_bounds__(kThreads) void k_filter_adjoint_scale(
    Geometry g, const double* __restrict__ rt, double rmin, double beta, Etas eta, int nsys,
    const double* __restrict__ gin, double* __restrict__ ge) {
  const int R = rmin > 1.0 ? (int)ceil(rmin) - 1 : 0;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < g.nel;
       e += (int64_t)gridDim.x * kThreads) {
    double den = 1.0;
    if (R > 0) {
      int ex, ey, ez;
      elem_coords(g, e, ex, ey, ez);
      den = weight_sum(g, ex, ey, ez, rmin, R);
    }
    const double x = rt[e];
    for (int s = 0; s < nsys; ++s)
      ge[(size_t)s * g.nel + e] = gin[(size_t)s * g.nel + e] * heaviside_d(x, beta, eta.v[s]) / den;
  }
}

// dc/drho_i = sum_{e near i} w_ie ge_e (the filter weights are symmetric)
__global__ __launch_bounds__(kThreads) void k_filter_project_adjoint(
    Geometry g, double rmin, int nsys, const double* __restrict__ ge, double* __restrict__ out) {
  const int R = rmin > 1.0 ? (int)ceil(rmin) - 1 : 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < g.nel;
       i += (int64_t)gridDim.x * kThreads) {
    double acc[kMaxSys] = {0.0, 0.0, 0.0, 0.0};
    if (R == 0) {
      for (int s = 0; s < nsys; ++s) acc[s] = ge[(size_t)s * g.nel + i];
    } else {
      int ix, iy, iz;
      elem_coords(g, i, ix, iy, iz);
      const int R3 = g.dim == 3 ? R : 0;
      for (int dz = -R3; dz <= R3; ++dz)
        for (int dy = -R; dy <= R; ++dy)
          for (int dx = -R; dx <= R; ++dx) {
            const int x = ix + dx, y = iy + dy, z = iz + dz;
            if (x < 0 || x >= g.nelx || y < 0 || y >= g.nely || z < 0 || z >= g.nelz) continue;
            const double w = rmin - sqrt((double)(dx * dx + dy * dy + dz * dz));
            if (w <= 0.0) continue;
            const int64_t e = x + (int64_t)g.nelx * (y + (int64_t)g.nely * z);
            for (int s = 0; s < nsys; ++s) acc[s] += w * ge[(size_t)s * g.nel + e];
          }
    }
    for (int s = 0; s < nsys; ++s) out[(size_t)s * g.nel + i] = acc[s];
  }
}

// D = g.dim as a constant: the element vector is indexed statically and
// stays in registers
template <int D>
__global__ __launch_bounds__(kThreads) void k_sensitivity(Geometry g, const double* __restrict__ rho,
                                                         const double* __restrict__ u,
                                                         const uint8_t* __restrict__ fixed,
                                                         const double* __restrict__ K0,
                                                         double E0, double Emin, double penal,
                                                         double* __restrict__ dc) {
  __shared__ double K0s[576];
  const int sys = blockIdx.y;
  constexpr int d = D, nd = D == 3 ? 24 : 8;
  for (int i = threadIdx.x; i < nd * nd; i += kThreads) K0s[i] = K0[i];
  __syncthreads();
  const double* us = u + (size_t)sys * g.ndof;
  const double* rs = rho + (size_t)sys * g.nel;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < g.nel;
       e += (int64_t)gridDim.x * kThreads) {
    int ex, ey, ez;
    elem_coords(g, e, ex, ey, ez);
    const int64_t n0 = ex + (int64_t)g.nnx * (ey + (int64_t)g.nny * ez);
    const int64_t lay = (int64_t)g.nnx * g.nny;
    int64_t nodes[8] = {n0, n0 + 1, n0 + 1 + g.nnx, n0 + g.nnx, 0, 0, 0, 0};
    constexpr int na = D == 3 ? 8 : 4;
    if (D == 3)
#pragma unroll
      for (int a = 0; a < 4; ++a) nodes[4 + a] = nodes[a] + lay;
    double ue[nd];
#pragma unroll
    for (int a = 0; a < na; ++a)
#pragma unroll
      for (int c = 0; c < d; ++c) {
        const int64_t dof = d * nodes[a] + c;
        ue[d * a + c] = fixed[dof] ? 0.0 : us[dof];
      }
    double q = 0.0;
#pragma unroll 1
    for (int a = 0; a < nd; ++a) {
      double t = 0.0, ua = 0.0;
#pragma unroll
      for (int b = 0; b < nd; ++b) {
        t += K0s[a * nd + b] * ue[b];
        ua = b == a ? ue[b] : ua;   // ue[a] without a dynamic register index
      }
      q += ua * t;
    }
    const double r = rs[e];
    const double rp1 = penal == 3.0 ? r * r : pow(r, penal - 1.0);
    dc[(size_t)sys * g.nel + e] = -penal * (E0 - Emin) * rp1 * q;
  }
}

// partials of f^T u over the free DOFs: part[sys * kMaxParts + workgroup]
__global__ __launch_bounds__(kThreads) void k_fu_parts(Geometry g, const double* __restrict__ f,
                                                      const double* __restrict__ u,
                                                      const uint8_t* __restrict__ fixed,
                                                      double* __restrict__ part) {
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  const size_t off = (size_t)sys * g.ndof;
  double a = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < g.nnodes;
       n += (int64_t)gridDim.x * kThreads)
    for (int c = 0; c < g.dim; ++c) {
      const int64_t i = g.dim * n + c;
      if (!fixed[i]) a += f[off + i] * u[off + i];
    }
  const double s = block_sum(a, sh);
  if (threadIdx.x == 0) part[(size_t)sys * kMaxParts + blockIdx.x] = s;
}

__global__ void k_fu_final(const double* __restrict__ part, int np, double* __restrict__ c) {
  __shared__ double sh[4];
  const int sys = blockIdx.x;
  const double v = sum_parts(part + (size_t)sys * kMaxParts, np, sh);
  if (threadIdx.x == 0) c[sys] = v;
}

// Robust objective of the realisations' compliances (Sec. 4.4): every
// thread forms the mean and the population standard deviation of c from the
// weights in the same order; out = {E[c] + kappa std, E[c], std} and
// df[i] = sum_s w_s (1 + kappa (c_s - E[c]) / std) dc[s][i] (no variance
// term when std = 0).
struct RobustW {
  double w[kMaxSys];
  double kappa;
};

__global__ __launch_bounds__(kThreads) void k_robust(const double* __restrict__ c,
                                                    const double* __restrict__ dc, int nsys,
                                                    int64_t n, RobustW rw, double* __restrict__ out,
                                                    double* __restrict__ df) {
  double mean = 0.0;
  for (int s = 0; s < nsys; ++s) mean += rw.w[s] * c[s];
  double var = 0.0;
  for (int s = 0; s < nsys; ++s) var += rw.w[s] * (c[s] - mean) * (c[s] - mean);
  const double sd = sqrt(var);
  double a[kMaxSys];
#pragma unroll
  for (int s = 0; s < kMaxSys; ++s)
    a[s] = s < nsys ? rw.w[s] * (1.0 + (sd > 0.0 ? rw.kappa * (c[s] - mean) / sd : 0.0)) : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out[0] = mean + rw.kappa * sd;
    out[1] = mean;
    out[2] = sd;
  }
  if (!dc) return;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double v = 0.0;
    for (int s = 0; s < nsys; ++s) v += a[s] * dc[(size_t)s * n + i];
    df[i] = v;
  }
}

// Sum over the periodic copies (Sec. 4.1): gcell[s][v] = sum of g[s][e] over
// the elements e at position v of the unit cell (cx, cy, cz), partial cells
// at the far faces included. One workgroup per (cell variable, system);
// copies summed in a fixed tree.
__global__ __launch_bounds__(kThreads) void k_periodic_sum(Geometry g, const double* __restrict__ gin,
                                                          int cx, int cy, int cz,
                                                          double* __restrict__ gcell) {
  __shared__ double sh[4];
  const int v = blockIdx.x, sys = blockIdx.y;
  const int vx = v % cx, vy = (v / cx) % cy, vz = v / (cx * cy);
  const int qx = (g.nelx + cx - 1) / cx, qy = (g.nely + cy - 1) / cy, qz = (g.nelz + cz - 1) / cz;
  const int64_t ncopy = (int64_t)qx * qy * qz;
  const double* gs = gin + (size_t)sys * g.nel;
  double acc = 0.0;
  for (int64_t q = threadIdx.x; q < ncopy; q += kThreads) {
    const int ax = (int)(q % qx), ay = (int)((q / qx) % qy), az = (int)(q / ((int64_t)qx * qy));
    const int ex = ax * cx + vx, ey = ay * cy + vy, ez = az * cz + vz;
    if (ex < g.nelx && ey < g.nely && ez < g.nelz)
      acc += gs[ex + (int64_t)g.nelx * (ey + (int64_t)g.nely * ez)];
  }
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) gcell[(size_t)sys * cx * cy * cz + v] = tot;
}

// partials of sum_e 4 rho_e (1 - rho_e) (the non-discreteness measure, Sec. 5.2)
__global__ __launch_bounds__(kThreads) void k_mnd_parts(const double* __restrict__ rho, int64_t n,
                                                       double* __restrict__ part) {
  __shared__ double sh[4];
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    a += 4.0 * rho[i] * (1.0 - rho[i]);
  const double s = block_sum(a, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_mnd_final(const double* __restrict__ part, int np, int64_t n,
                            double* __restrict__ out) {
  __shared__ double sh[4];
  const double v = sum_parts(part, np, sh);
  if (threadIdx.x == 0) out[0] = v / (double)n;
}

int elem_blocks(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

void launch_filter_project(const Handle& h, const double* rho, double rmin, double beta,
                           const double* eta, int nsys, double* rho_tilde, double* rho_phys,
                           hipStream_t st) {
  Etas e{};
  for (int s = 0; s < nsys; ++s) e.v[s] = eta[s];
  hipLaunchKernelGGL(k_filter_project, dim3(elem_blocks(h.g.nel)), dim3(kThreads), 0, st, h.g,
                     rho, rmin, beta, e, nsys, rho_tilde, rho_phys);
}

void launch_filter_project_adjoint(const Handle& h, const double* rho_tilde, double rmin,
                                   double beta, const double* eta, int nsys, const double* g,
                                   double* out, hipStream_t st) {
  Etas e{};
  for (int s = 0; s < nsys; ++s) e.v[s] = eta[s];
  hipLaunchKernelGGL(k_filter_adjoint_scale, dim3(elem_blocks(h.g.nel)), dim3(kThreads), 0, st,
                     h.g, rho_tilde, rmin, beta, e, nsys, g, h.fscratch);
  hipLaunchKernelGGL(k_filter_project_adjoint, dim3(elem_blocks(h.g.nel)), dim3(kThreads), 0, st,
                     h.g, rmin, nsys, h.fscratch, out);
}

void launch_robust(const Handle& h, const double* c, const double* dc, int nsys, double kappa,
                   const double* w, double* out, double* df, hipStream_t st) {
  RobustW rw{};
  for (int s = 0; s < nsys; ++s) rw.w[s] = w[s];
  rw.kappa = kappa;
  hipLaunchKernelGGL(k_robust, dim3(dc ? elem_blocks(h.g.nel) : 1), dim3(kThreads), 0, st, c, dc,
                     nsys, (int64_t)h.g.nel, rw, out, df);
}

void launch_periodic_sum(const Handle& h, const double* gin, int nsys, int cx, int cy, int cz,
                         double* gcell, hipStream_t st) {
  hipLaunchKernelGGL(k_periodic_sum, dim3(cx * cy * cz, nsys), dim3(kThreads), 0, st, h.g, gin, cx,
                     cy, cz, gcell);
}

void launch_nondiscreteness(const Handle& h, const double* rho, double* out, hipStream_t st) {
  const int np = parts_for(h.g.nel);
  double* part = part_slot(h.parts, kPartAux, 0);
  hipLaunchKernelGGL(k_mnd_parts, dim3(np), dim3(kThreads), 0, st, rho, (int64_t)h.g.nel, part);
  hipLaunchKernelGGL(k_mnd_final, dim3(1), dim3(kThreads), 0, st, part, np, (int64_t)h.g.nel, out);
}

void launch_compliance_sens_raw(const Geometry& g, const uint8_t* fixed, const double* K0,
                                double E0, double Emin, double penal, double* part,
                                const double* rho, const double* u, const double* f, int nsys,
                                double* c, double* dc, hipStream_t st) {
  const int np = parts_for(g.nnodes);
  hipLaunchKernelGGL(k_fu_parts, dim3(np, nsys), dim3(kThreads), 0, st, g, f, u, fixed, part);
  hipLaunchKernelGGL(k_fu_final, dim3(nsys), dim3(kThreads), 0, st, part, np, c);
  if (dc) {
    if (g.dim == 2)
      hipLaunchKernelGGL(k_sensitivity<2>, dim3(elem_blocks(g.nel), nsys), dim3(kThreads), 0, st,
                         g, rho, u, fixed, K0, E0, Emin, penal, dc);
    else
      hipLaunchKernelGGL(k_sensitivity<3>, dim3(elem_blocks(g.nel), nsys), dim3(kThreads), 0, st,
                         g, rho, u, fixed, K0, E0, Emin, penal, dc);
  }
}

void launch_compliance_sens(const Handle& h, const double* rho, const double* u, const double* f,
                            int nsys, double* c, double* dc, hipStream_t st) {
  const tpcg_problem& pr = h.prob;
  launch_compliance_sens_raw(h.g, h.fixed, h.K0, pr.E0, pr.Emin, pr.penal,
                             part_slot(h.parts, kPartAux, 0), rho, u, f, nsys, c, dc, st);
}

}  // namespace tpcg
