// Batched PCG vector kernels with fused, deterministic reductions.
//
// Each kernel sweeps all DOFs of a system with parts_for(nnodes) workgroups,
// one node per thread per step, and writes one partial sum per workgroup.
// Scalars (alpha, beta, convergence) are recomputed by every consumer from
// those partials in a fixed order, so no workgroup ever waits for another and
// all of them agree bit for bit. Systems that have converged are masked.
#include "tpcg_internal.h"

namespace tpcg {

namespace {

// r = P (f - q), u <- P u; partials of r.r (slot RR0) and (Pf).(Pf) (slot FF).
__global__ __launch_bounds__(kThreads) void k_residual_init(
    Geometry g, const double* __restrict__ f, double* __restrict__ u,
    const double* __restrict__ q, double* __restrict__ r, const uint8_t* __restrict__ fixed,
    double* __restrict__ parts, int* __restrict__ istate) {
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  const int d = g.dim;
  const size_t off = (size_t)sys * g.ndof;
  double arr = 0.0, aff = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < g.nnodes;
       n += (int64_t)gridDim.x * kThreads) {
    for (int c = 0; c < d; ++c) {
      const size_t i = off + d * n + c;
      const bool fx = fixed[d * n + c];
      const double fi = fx ? 0.0 : f[i];
      const double ri = fx ? 0.0 : fi - q[i];
      r[i] = ri;
      if (fx) u[i] = 0.0;
      arr += ri * ri;
      aff += fi * fi;
    }
  }
  const double srr = block_sum(arr, sh);
  const double sff = block_sum(aff, sh);
  if (threadIdx.x == 0) {
    part_slot(parts, kPartRR0, sys)[blockIdx.x] = srr;
    part_slot(parts, kPartFF, sys)[blockIdx.x] = sff;
    if (blockIdx.x == 0) {
      istate[kStLastIt * kMaxSys + sys] = 0;
      istate[kStBreak * kMaxSys + sys] = 0;
      if (sys == 0) istate[kStIter * kMaxSys] = 0;
    }
  }
}

// Iteration `it`: alpha = (r.z)/(p.q) (r.z from the scalar slot, np_pq
// partials of p.q from the operator launch); u += alpha p; r -= alpha q;
// partials of the new r.r into the other parity slot. Breakdown (p.q <= 0
// or not finite) stops the system.
__global__ __launch_bounds__(kThreads) void k_update_xr(
    Geometry g, double* __restrict__ u, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, double* __restrict__ parts, int* __restrict__ istate,
    Gate gate, int np_pq) {
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  const int slot_old = gate.rr_slot;
  const int slot_new = slot_old == kPartRR0 ? kPartRR1 : kPartRR0;
  bool run = gate_running(gate, sys);
  const int d = g.dim;
  const size_t off = (size_t)sys * g.ndof;
  // the first node's loads go out before alpha is reduced, so that their
  // latency overlaps the reduction
  const int64_t n0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool has0 = run && n0 < g.nnodes;
  double u0[3], p0[3], r0[3], q0[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    u0[c] = p0[c] = r0[c] = q0[c] = 0.0;
    if (has0 && c < d) {
      const size_t i = off + d * n0 + c;
      u0[c] = u[i];
      p0[c] = p[i];
      r0[c] = r[i];
      q0[c] = q[i];
    }
  }
  double alpha = 0.0;
  if (run) {
    const double pq = sum_parts(part_slot(parts, kPartPQ, sys), np_pq, sh);
    const double rz = scal_slot(parts, kScRZ)[sys];
    alpha = rz / pq;
    if (!(pq > 0.0) || !isfinite(alpha)) {
      run = false;
      if (blockIdx.x == 0 && threadIdx.x == 0) istate[kStBreak * kMaxSys + sys] = 1;
    }
  }
  if (!run) {
    if (threadIdx.x == 0)
      part_slot(parts, slot_new, sys)[blockIdx.x] = part_slot(parts, slot_old, sys)[blockIdx.x];
    return;
  }
  double arr = 0.0;
  if (has0) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (c < d) {
        const size_t i = off + d * n0 + c;
        u[i] = u0[c] + alpha * p0[c];
        const double ri = r0[c] - alpha * q0[c];
        r[i] = ri;
        arr += ri * ri;
      }
  }
  for (int64_t n = n0 + (int64_t)gridDim.x * kThreads; n < g.nnodes;
       n += (int64_t)gridDim.x * kThreads) {
    for (int c = 0; c < d; ++c) {
      const size_t i = off + d * n + c;
      u[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      arr += ri * ri;
    }
  }
  const double s = block_sum(arr, sh);
  if (threadIdx.x == 0) {
    part_slot(parts, slot_new, sys)[blockIdx.x] = s;
    if (blockIdx.x == 0) istate[kStLastIt * kMaxSys + sys] = gate_it(gate) + 1;
  }
}

// One workgroup per system, after the preconditioner of iteration `it` (the
// gate refers to the residual after that iteration's update): r.z_new from
// its partials; beta = (r.z_new)/(r.z_old), or the flexible (Polak-Ribiere)
// form (r.z_new - r.z_prev)/(r.z_old) when the preconditioner is not exactly
// symmetric (FP32 inner solves); first: beta = 0. r.z_new replaces r.z_old.
__global__ __launch_bounds__(kThreads) void k_beta(Gate gate, int rz_slot, int flexible, int first,
                                                   int* __restrict__ istate) {
  __shared__ double sh[4];
  const int sys = blockIdx.x;
  if (!gate_running(gate, sys)) return;
  double* parts = const_cast<double*>(gate.parts);
  const double rzn = sum_parts(part_slot(parts, rz_slot, sys), gate.np, sh);
  double beta = 0.0;
  bool brk = false;
  if (!first) {
    double num = rzn;
    if (flexible) num -= sum_parts(part_slot(parts, kPartRZO, sys), gate.np, sh);
    beta = num / scal_slot(parts, kScRZ)[sys];
    brk = !(rzn > 0.0) || !isfinite(beta);
  }
  if (threadIdx.x == 0) {
    if (brk) istate[kStBreak * kMaxSys + sys] = 1;
    scal_slot(parts, kScBeta)[sys] = beta;
    scal_slot(parts, kScRZ)[sys] = rzn;
  }
}

// the residual test of the gate, once per iteration: kStRun = r.r > tol2 ||Pf||^2
__global__ __launch_bounds__(kThreads) void k_gate(Gate gate, int* __restrict__ istate) {
  __shared__ double sh[4];
  const int sys = blockIdx.x;
  double* parts = const_cast<double*>(gate.parts);
  const double rr = sum_parts(part_slot(parts, gate.rr_slot, sys), gate.np, sh);
  const double ff = sum_parts(part_slot(parts, kPartFF, sys), gate.np, sh);
  if (threadIdx.x == 0) {
    istate[kStRun * kMaxSys + sys] = rr > gate.tol2 * ff ? 1 : 0;
    scal_slot(parts, kScFF)[sys] = ff;   // for the tests taken inside kernels
  }
}

__global__ void k_poll(Gate gate, int* __restrict__ istate, int advance) {
  const int sys = blockIdx.x;
  const bool run = gate_running(gate, sys);
  if (threadIdx.x == 0) {
    istate[kStPoll * kMaxSys + sys] = run ? 1 : 0;
    if (sys == 0) istate[kStIter * kMaxSys] += advance;
  }
}

// flag[sys * stride] = value when a density of system sys is NaN or outside
// [0, 1] (racing writers store the same value)
__global__ __launch_bounds__(kThreads) void k_check_rho(const double* __restrict__ rho, int64_t n,
                                                       int* __restrict__ flag, int stride,
                                                       int value) {
  const int sys = blockIdx.y;
  const double* rs = rho + (size_t)sys * n;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double v = rs[i];
    bad |= !(v >= 0.0 && v <= 1.0);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) flag[sys * stride] = value;
}

// partials of ||P (f - q)||^2 into slot Aux
__global__ __launch_bounds__(kThreads) void k_true_residual(
    Geometry g, const double* __restrict__ f, const double* __restrict__ q,
    const uint8_t* __restrict__ fixed, double* __restrict__ parts) {
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  const size_t off = (size_t)sys * g.ndof;
  double a = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < g.nnodes;
       n += (int64_t)gridDim.x * kThreads) {
    for (int c = 0; c < g.dim; ++c) {
      const size_t i = g.dim * n + c;
      const double v = fixed[i] ? 0.0 : f[off + i] - q[off + i];
      a += v * v;
    }
  }
  const double s = block_sum(a, sh);
  if (threadIdx.x == 0) part_slot(parts, kPartAux, sys)[blockIdx.x] = s;
}

// out[sys] = {iterations, status, relres, true_relres}
__global__ void k_finalize(Gate gate, const double* __restrict__ parts,
                           const int* __restrict__ istate, double* __restrict__ out) {
  __shared__ double sh[4];
  const int sys = blockIdx.x;
  const double rr = sum_parts(part_slot(const_cast<double*>(parts), gate.rr_slot, sys), gate.np, sh);
  const double ff = sum_parts(part_slot(const_cast<double*>(parts), kPartFF, sys), gate.np, sh);
  const double tr = sum_parts(part_slot(const_cast<double*>(parts), kPartAux, sys), gate.np, sh);
  if (threadIdx.x == 0) {
    const int brk = istate[kStBreak * kMaxSys + sys];
    double status = TPCG_OK;
    if (brk == 2) status = TPCG_EINVAL;
    else if (brk) status = TPCG_EBREAKDOWN;
    else if (!(rr <= gate.tol2 * ff)) status = TPCG_ENOCONV;
    out[4 * sys + 0] = istate[kStLastIt * kMaxSys + sys];
    out[4 * sys + 1] = status;
    out[4 * sys + 2] = ff > 0.0 ? sqrt(rr / ff) : 0.0;
    out[4 * sys + 3] = ff > 0.0 ? sqrt(tr / ff) : 0.0;
  }
}

}  // namespace

void launch_residual_init(const Handle& h, const double* f, double* u, const double* q, int nsys,
                          hipStream_t st) {
  dim3 grid(parts_for(h.g.nnodes), nsys);
  hipLaunchKernelGGL(k_residual_init, grid, dim3(kThreads), 0, st, h.g, f, u, q, h.r, h.fixed,
                     h.parts, h.istate);
}

void launch_update_xr(const Handle& h, double* u, const double* p, int nsys, const Gate& gate,
                      hipStream_t st) {
  dim3 grid(parts_for(h.g.nnodes), nsys);
  hipLaunchKernelGGL(k_update_xr, grid, dim3(kThreads), 0, st, h.g, u, h.r, p, h.q, h.parts,
                     h.istate, gate, apply_parts(h.g));
}

void launch_beta(const Handle& h, int nsys, const Gate& gate, int rz_slot, int flexible,
                 int first, hipStream_t st) {
  hipLaunchKernelGGL(k_beta, dim3(nsys), dim3(kThreads), 0, st, gate, rz_slot, flexible, first,
                     h.istate);
}

void launch_gate(const Handle& h, int nsys, const Gate& gate, hipStream_t st) {
  hipLaunchKernelGGL(k_gate, dim3(nsys), dim3(kThreads), 0, st, gate, h.istate);
}

void launch_poll(const Handle& h, int nsys, const Gate& gate, int advance, hipStream_t st) {
  hipLaunchKernelGGL(k_poll, dim3(nsys), dim3(kThreads), 0, st, gate, h.istate, advance);
}

void launch_check_rho(const double* rho, int64_t n, int nsys, int* flag, int stride, int value,
                      hipStream_t st) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_check_rho, dim3((unsigned)b, nsys), dim3(kThreads), 0, st, rho, n, flag,
                     stride, value);
}

void launch_copy(double* dst, const double* src, int64_t n, hipStream_t st) {
  hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
}

// True residual and the per-system summary; q must already hold K u.
void launch_summary(const Handle& h, const double* f, int nsys, const Gate& gate, double* out,
                    hipStream_t st) {
  dim3 grid(parts_for(h.g.nnodes), nsys);
  hipLaunchKernelGGL(k_true_residual, grid, dim3(kThreads), 0, st, h.g, f, h.q, h.fixed, h.parts);
  hipLaunchKernelGGL(k_finalize, dim3(nsys), dim3(kThreads), 0, st, gate, h.parts, h.istate, out);
}

}  // namespace tpcg
