// Matrix-free stiffness product y = P K(rho) P x (Sec. 2.1 discrete system,
// Sec. 2.2 element stiffness K_e = (E_min + (E0 - E_min) rho_e^p) K0).
//
// Each node's row is gathered from the node's elements: for each element e
// around the node, the rows of E_e K0 that belong to the node times the
// element's nodal displacements. No atomics; each output is written once.
// K0 lives in LDS; the SIMP modulus is evaluated in the kernel.
#include <algorithm>

#include "tpcg_internal.h"

namespace tpcg {

namespace {

// Q4: the mesh is cut into tiles of kTX x kTY nodes. A workgroup stages the
// tile's halo of P x (one node ring, rows contiguous in memory) and the moduli
// of the tile's elements in LDS, then each thread forms two nodes' rows of
// y = P K P x from LDS only, so x and rho are read from HBM about once.
constexpr int kTX = 64, kTY = 8;
constexpr int kHX = kTX + 2, kHY = kTY + 2;   // halo of nodes
constexpr int kEX = kTX + 1, kEY = kTY + 1;   // elements touching the tile

__host__ __device__ inline int q4_tiles(const Geometry& g) {
  return ((g.nnx + kTX - 1) / kTX) * ((g.nny + kTY - 1) / kTY);
}

__global__ __launch_bounds__(kThreads) void k_apply_q4(
    Geometry g, const double* __restrict__ rho, const double* __restrict__ x,
    double* __restrict__ y, const uint8_t* __restrict__ fixed, const double* __restrict__ K0,
    double E0, double Emin, double penal, double* __restrict__ parts, Gate gate) {
  __shared__ double K0s[64];
  __shared__ double2 xh[kHY * kHX];
  __shared__ double Eh[kEY * kEX];
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  const int t = threadIdx.x;
  if (t < 64) K0s[t] = K0[t];
  const double* xs = x + (size_t)sys * g.ndof;
  double* ys = y + (size_t)sys * g.ndof;
  const double* rs = rho + (size_t)sys * g.nel;
  const uint16_t* fx2 = reinterpret_cast<const uint16_t*>(fixed);   // both flags of a node
  const int nnx = g.nnx, nny = g.nny;
  const int ntx = (nnx + kTX - 1) / kTX, ntiles = q4_tiles(g);
  const int tx = t % kTX, ty = t / kTX;   // kThreads / kTX = 4 rows of threads
  double acc = 0.0;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % ntx) * kTX, y0 = (tile / ntx) * kTY;
    __syncthreads();   // the previous tile's LDS reads are done
    for (int i = t; i < kHY * kHX; i += kThreads) {
      const int X = x0 - 1 + i % kHX, Y = y0 - 1 + i / kHX;
      double2 v = make_double2(0.0, 0.0);
      if (X >= 0 && X < nnx && Y >= 0 && Y < nny) {
        const int64_t n = X + (int64_t)nnx * Y;
        v = *reinterpret_cast<const double2*>(xs + 2 * n);
        const uint16_t f = fx2[n];
        if (f & 0x00ffu) v.x = 0.0;
        if (f & 0xff00u) v.y = 0.0;
      }
      xh[i] = v;
    }
    for (int i = t; i < kEY * kEX; i += kThreads) {
      const int ex = x0 - 1 + i % kEX, ey = y0 - 1 + i / kEX;
      double E = 0.0;
      if (ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely)
        E = simp_modulus(rs[ex + (int64_t)g.nelx * ey], E0, Emin, penal);
      Eh[i] = E;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const int lx = tx, ly = ty + 4 * rr;              // tile-local node
      const int X = x0 + lx, Y = y0 + ly;
      if (X >= nnx || Y >= nny) continue;
      double y0v = 0.0, y1v = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        // the node is corner a of element (ex, ey); corners counter-clockwise
        const int dx = (a == 1) || (a == 2), dy = a >= 2;
        const double E = Eh[(ly - dy + 1) * kEX + (lx - dx + 1)];
        const int hx0 = lx - dx + 1, hy0 = ly - dy + 1;  // halo index of the element's corner 0
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int bx = (b == 1) || (b == 2), by = b >= 2;
          const double2 u = xh[(hy0 + by) * kHX + hx0 + bx];
          t0 += K0s[(2 * a) * 8 + 2 * b] * u.x + K0s[(2 * a) * 8 + 2 * b + 1] * u.y;
          t1 += K0s[(2 * a + 1) * 8 + 2 * b] * u.x + K0s[(2 * a + 1) * 8 + 2 * b + 1] * u.y;
        }
        y0v += E * t0;
        y1v += E * t1;
      }
      const int64_t n = X + (int64_t)nnx * Y;
      const uint16_t f = fx2[n];
      if (f & 0x00ffu) y0v = 0.0;
      if (f & 0xff00u) y1v = 0.0;
      *reinterpret_cast<double2*>(ys + 2 * n) = make_double2(y0v, y1v);
      if (parts) {
        const double2 xv = xh[(ly + 1) * kHX + lx + 1];   // already P x
        acc += xv.x * y0v + xv.y * y1v;
      }
    }
  }
  if (parts) {
    const double v = block_sum(acc, sh);
    if (t == 0) parts[(size_t)sys * kMaxParts + blockIdx.x] = v;
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

int apply_parts(const Geometry& g) {
  if (g.dim == 2) return std::min(q4_tiles(g), kMaxParts);
  return parts_for(g.nnodes);
}

void launch_apply_K(const Handle& h, const double* rho, const double* x, double* y, int nsys,
                    int dot_slot, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  dim3 grid(apply_parts(g), nsys);
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
