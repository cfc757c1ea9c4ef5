// Matrix-free stiffness product y = P K(rho) P x (Sec. 2.1 discrete system,
// Sec. 2.2 element stiffness K_e = (E_min + (E0 - E_min) rho_e^p) K0).
//
// Each node's row is gathered from the node's elements: for each element e
// around the node, the rows of E_e K0 that belong to the node times the
// element's nodal displacements. No atomics; each output is written once.
// K0 lives in LDS; the SIMP modulus is evaluated in the kernel.
#include <algorithm>
#include <cmath>

#include "tpcg_internal.h"

namespace tpcg {

namespace {

// Q4: the mesh is cut into tiles of kTX x kTY nodes. A workgroup stages the
// tile's halo of P x (one node ring, rows contiguous in memory) and the moduli
// of the elements touching the tile in LDS; thread (tx, ty) then forms the
// rows of y = P K P x for the kRN nodes of column tx, rows kRN ty ..
// kRN ty + kRN - 1, sliding a 3 x 3 window of nodal values and a 2 x 2
// window of moduli down the column.
//
// The unit-square bilinear element matrix has only eight distinct entries
// (the square's reflections and its rotation by a right angle map each entry
// to one of them): K0 = q[kQ4Map], q its first row. q is uniform over the
// launch and passed by value, so K0 comes from scalar registers and the LDS
// carries only the nodal values and moduli.
constexpr int kTX = 64, kRN = 4, kTY = (kThreads / kTX) * kRN;
constexpr int kHX = kTX + 2, kHY = kTY + 2;   // halo of nodes
constexpr int kEX = kTX + 1, kEY = kTY + 1;   // elements touching the tile

constexpr int kQ4Map[8][8] = {{0, 1, 2, 3, 4, 5, 6, 7}, {1, 0, 7, 6, 5, 4, 3, 2},
                              {2, 7, 0, 5, 6, 3, 4, 1}, {3, 6, 5, 0, 7, 2, 1, 4},
                              {4, 5, 6, 7, 0, 1, 2, 3}, {5, 4, 3, 2, 1, 0, 7, 6},
                              {6, 3, 4, 1, 2, 7, 0, 5}, {7, 2, 1, 4, 3, 6, 5, 0}};

struct Q4Row {
  double q[8];
};

__host__ __device__ inline int q4_tiles(const Geometry& g) {
  return ((g.nnx + kTX - 1) / kTX) * ((g.nny + kTY - 1) / kTY);
}

// P3: penal == 3, the modulus without pow (whose code would otherwise hold
// registers through the whole kernel)
//
// DIR: the CG direction update is fused in: the product is taken with
// p = z + beta p_old (p = z when first), formed for the staged halo from z
// and p_old = x, and the workgroup writes p for the nodes it owns to pnew
// (a buffer other than x, since neighbouring tiles still read p_old).
template <bool P3, bool DIR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_apply_q4(
    Geometry g, const double* __restrict__ rho, const double* __restrict__ x,
    double* __restrict__ y, const uint8_t* __restrict__ fixed, Q4Row K, double E0, double Emin,
    double penal, double* __restrict__ parts, Gate gate, const double* __restrict__ zdir,
    double* __restrict__ pnew, const double* __restrict__ beta, int first) {
  constexpr int kHN = (kHY * kHX + kThreads - 1) / kThreads;   // staged values per thread
  constexpr int kEN = (kEY * kEX + kThreads - 1) / kThreads;
  __shared__ double2 xh[kHY * kHX];
  __shared__ double Eh[kEY * kEX];
  __shared__ double sh[4];
  const int nnx = g.nnx, nny = g.nny;
  const int ntx = (nnx + kTX - 1) / kTX, ntiles = q4_tiles(g);
  // XCD-aware order: workgroups go to the chip's 8 XCDs in turn, so those
  // of one system whose index agrees mod 8 share an XCD. With one tile per
  // workgroup the remap below gives each such group a contiguous range of
  // the system's tiles, whose shared halo lines then meet in that XCD's L2;
  // every system still spreads over all XCDs
  const int sys = blockIdx.y;
  int slot = blockIdx.x;
  if (gridDim.x == ntiles) {
    const int W = gridDim.x, w = blockIdx.x;
    const int grp = w % 8, k = w / 8, per = W / 8, rem = W % 8;
    slot = (grp < rem ? grp * (per + 1) : rem * (per + 1) + (grp - rem) * per) + k;
  }
  if (!gate_running(gate, sys)) return;
  const int t = threadIdx.x;
  const double* xs = x + (size_t)sys * g.ndof;
  double* ys = y + (size_t)sys * g.ndof;
  const double* rs = rho + (size_t)sys * g.nel;
  const double* zs = DIR ? zdir + (size_t)sys * g.ndof : nullptr;
  double* ps = DIR ? pnew + (size_t)sys * g.ndof : nullptr;
  const double bt = DIR && !first ? beta[sys] : 0.0;
  const uint16_t* fx2 = reinterpret_cast<const uint16_t*>(fixed);   // both flags of a node
  const int tx = t % kTX, ty = t / kTX;
  double acc = 0.0;
  for (int tile = slot; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % ntx) * kTX, y0 = (tile / ntx) * kTY;
    // every load of the tile is issued before any is used
    double2 hv[kHN];
    uint16_t hf[kHN];
    double rv[kEN];
#pragma unroll
    for (int q = 0; q < kHN; ++q) {
      const int i = t + q * kThreads;
      const int X = x0 - 1 + i % kHX, Y = y0 - 1 + i / kHX;
      hv[q] = make_double2(0.0, 0.0);
      hf[q] = 0xffffu;
      if (i < kHY * kHX && X >= 0 && X < nnx && Y >= 0 && Y < nny) {
        const int64_t n = X + (int64_t)nnx * Y;
        if (DIR) {
          const double2 zv = *reinterpret_cast<const double2*>(zs + 2 * n);
          double2 pv = make_double2(0.0, 0.0);
          if (!first) pv = *reinterpret_cast<const double2*>(xs + 2 * n);
          hv[q] = make_double2(zv.x + bt * pv.x, zv.y + bt * pv.y);
        } else {
          hv[q] = *reinterpret_cast<const double2*>(xs + 2 * n);
        }
        hf[q] = fx2[n];
      }
    }
#pragma unroll
    for (int q = 0; q < kEN; ++q) {
      const int i = t + q * kThreads;
      const int ex = x0 - 1 + i % kEX, ey = y0 - 1 + i / kEX;
      rv[q] = -1.0;   // outside the mesh
      if (i < kEY * kEX && ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely)
        rv[q] = rs[ex + (int64_t)g.nelx * ey];
    }
    __syncthreads();   // the previous tile's LDS reads are done
#pragma unroll
    for (int q = 0; q < kHN; ++q) {
      const int i = t + q * kThreads;
      double2 v = hv[q];
      if (hf[q] & 0x00ffu) v.x = 0.0;
      if (hf[q] & 0xff00u) v.y = 0.0;
      if (i < kHY * kHX) xh[i] = v;
    }
#pragma unroll
    for (int q = 0; q < kEN; ++q) {
      const int i = t + q * kThreads;
      const double r = rv[q];
      const double E = r < 0.0 ? 0.0
                               : (P3 ? Emin + (E0 - Emin) * (r * r * r)
                                     : simp_modulus(r, E0, Emin, penal));
      if (i < kEY * kEX) Eh[i] = E;
    }
    __syncthreads();
    // window rows: halo rows kRN ty + i .. + 2, element rows kRN ty + i .. + 1
    double2 w[3][3];
    double e[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) w[r + 1][c] = xh[(kRN * ty + r) * kHX + tx + c];
#pragma unroll
    for (int c = 0; c < 2; ++c) e[1][c] = Eh[kRN * ty * kEX + tx + c];
#pragma unroll
    for (int i = 0; i < kRN; ++i) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[0][c] = w[1][c];
        w[1][c] = w[2][c];
        w[2][c] = xh[(kRN * ty + i + 2) * kHX + tx + c];
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        e[0][c] = e[1][c];
        e[1][c] = Eh[(kRN * ty + i + 1) * kEX + tx + c];
      }
      double y0v = 0.0, y1v = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        // the node (window row 1, column 1) is corner a of the element whose
        // corner 0 is window (1 - dy, 1 - dx); corners counter-clockwise
        const int dx = (a == 1) || (a == 2), dy = a >= 2;
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int bx = (b == 1) || (b == 2), by = b >= 2;
          const double2 u = w[1 - dy + by][1 - dx + bx];
          t0 += K.q[kQ4Map[2 * a][2 * b]] * u.x + K.q[kQ4Map[2 * a][2 * b + 1]] * u.y;
          t1 += K.q[kQ4Map[2 * a + 1][2 * b]] * u.x + K.q[kQ4Map[2 * a + 1][2 * b + 1]] * u.y;
        }
        const double E = e[1 - dy][1 - dx];
        y0v += E * t0;
        y1v += E * t1;
      }
      const int X = x0 + tx, Y = y0 + kRN * ty + i;
      if (X < nnx && Y < nny) {
        const int64_t n = X + (int64_t)nnx * Y;
        const uint16_t f = fx2[n];
        if (f & 0x00ffu) y0v = 0.0;
        if (f & 0xff00u) y1v = 0.0;
        *reinterpret_cast<double2*>(ys + 2 * n) = make_double2(y0v, y1v);
        if (DIR) *reinterpret_cast<double2*>(ps + 2 * n) = w[1][1];   // the new p
        if (parts) acc += w[1][1].x * y0v + w[1][1].y * y1v;   // w[1][1]: P x at the node
      }
      __builtin_amdgcn_sched_barrier(0);   // one node at a time: fewer live registers
    }
  }
  if (parts) {
    const double v = block_sum(acc, sh);
    if (t == 0) parts[(size_t)sys * kMaxParts + slot] = v;
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

bool q4_structured(const double* K0) {
  double mx = 0.0;
  for (int i = 0; i < 64; ++i) mx = std::max(mx, std::fabs(K0[i]));
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j)
      if (std::fabs(K0[8 * i + j] - K0[kQ4Map[i][j]]) > 1e-14 * mx) return false;
  return true;
}

int apply_parts(const Geometry& g) {
  if (g.dim == 2) return std::min(q4_tiles(g), kMaxParts);
  return parts_for(g.nnodes);
}

void launch_apply_K(const Handle& h, const double* rho, const double* x, double* y, int nsys,
                    int dot_slot, const Gate& gate, hipStream_t st) {
  launch_apply_K_dir(h, rho, nullptr, x, nullptr, y, nsys, dot_slot, gate, 0, st);
}

void launch_apply_K_dir(const Handle& h, const double* rho, const double* z, const double* x,
                        double* pnew, double* y, int nsys, int dot_slot, const Gate& gate,
                        int first, hipStream_t st) {
  const Geometry& g = h.g;
  dim3 grid(apply_parts(g), nsys);
  double* parts = dot_slot >= 0 ? part_slot(h.parts, dot_slot, 0) : nullptr;
  const double* beta = scal_slot(h.parts, kScBeta);
  const tpcg_problem& pr = h.prob;
  if (g.dim == 2) {
    Q4Row q;
    std::copy(h.K0q4, h.K0q4 + 8, q.q);
#define TPCG_Q4(P3, DIR)                                                                      \
  hipLaunchKernelGGL((k_apply_q4<P3, DIR>), grid, dim3(kThreads), 0, st, g, rho, x, y, h.fixed, \
                     q, pr.E0, pr.Emin, pr.penal, parts, gate, z, pnew, beta, first)
    if (z) {
      if (pr.penal == 3.0) TPCG_Q4(true, true);
      else TPCG_Q4(false, true);
    } else {
      if (pr.penal == 3.0) TPCG_Q4(true, false);
      else TPCG_Q4(false, false);
    }
#undef TPCG_Q4
  } else {
    hipLaunchKernelGGL(k_apply_h8, grid, dim3(kThreads), 0, st, g, rho, x, y, h.fixed, h.K0,
                       pr.E0, pr.Emin, pr.penal, parts, gate);
  }
}

}  // namespace tpcg
