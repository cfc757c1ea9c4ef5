// Matrix-free stiffness product y = P K(rho) P x (Sec. 2.1 discrete system,
// Sec. 2.2 element stiffness K_e = (E_min + (E0 - E_min) rho_e^p) K0).
//
// Each node's row is gathered from the node's elements: for each element e
// around the node, the rows of E_e K0 that belong to the node times the
// element's nodal displacements. No atomics; each output is written once.
// Both kernels stage a tile's halo in LDS and take K0 from scalar registers
// (the element matrices' symmetry leaves eight distinct entries in 2-d and
// twelve classes in 3-d); the SIMP modulus is evaluated in the kernel.
#include <algorithm>
#include <cmath>
#include <utility>

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

// H8: the mesh is cut into tiles of kBX x kBY x kBZ nodes, one node per
// thread (a wave is one z-layer of the tile). A workgroup stages the tile's
// one-node halo of P x in LDS, component-major so that the lanes of a wave
// read consecutive doubles, and the moduli of the elements touching the tile
// (zero outside the mesh, as are the halo values there). A thread then takes
// its node's 27 neighbours in turn: it reads the neighbour's three values once
// and adds them into t_a, the partial row of the node as corner a of each of
// its 8 elements that also holds the neighbour; the row is sum_a E_a t_a.
//
// The trilinear unit-cube matrix has twelve classes of entries. Reflect the
// element so that corner a goes to corner 0: corner b goes to the corner e
// with e_j = |p_b,j - p_a,j| (p: the corner's position), and the displacement
// components along the reflected axes change sign. So
//   K0[(a,i),(b,c)] = tau_i(a) tau_c(a) R(e)[i][c],  tau_j(a) = -1 if p_a,j = 1,
// where R(e) is the block of corner 0's rows. The axis permutations fix
// corner 0, and with the symmetry of K0 they leave twelve values in R, up to
// sign (h8_class). Class and sign are compile-time functions of the loop
// counters; the twelve values are uniform over the launch and passed by
// value, so every product reads K0 from scalar registers.
constexpr int kBX = 16, kBY = 4, kBZ = 4;                        // nodes per tile
constexpr int kGX = kBX + 2, kGY = kBY + 2, kGZ = kBZ + 2;       // halo of nodes
constexpr int kFX = kBX + 1, kFY = kBY + 1, kFZ = kBZ + 1;       // elements touching it
constexpr int kGN = kGX * kGY * kGZ, kGV = 3 * kGN, kFN = kFX * kFY * kFZ;
static_assert(kBX * kBY * kBZ == kThreads, "one node per thread");

struct H8Row {
  double q[12];
};

struct H8Cls {
  int q, s;   // class and sign
};

// class and sign of R(e)[i][c], e given as its three bits
__host__ __device__ constexpr H8Cls h8_class(int ex, int ey, int ez, int i, int c) {
  const int ei = i == 0 ? ex : (i == 1 ? ey : ez);
  const int ec = c == 0 ? ex : (c == 1 ? ey : ez);
  const int n1 = ex + ey + ez;
  if (n1 == 0) return {i == c ? 0 : 1, 1};
  if (n1 == 3) return {i == c ? 10 : 11, 1};
  if (n1 == 1) {   // b along one edge from a
    if (i == c) return {ei ? 2 : 3, 1};
    if (ei) return {4, 1};
    if (ec) return {4, -1};
    return {5, 1};
  }
  // b across a face from a
  if (i == c) return {ei ? 6 : 7, 1};
  if (ei && ec) return {8, 1};
  return {9, ec ? -1 : 1};
}

__host__ __device__ constexpr int corner_bit(int a, int j) {
  return j == 0 ? ((a & 3) == 1 || (a & 3) == 2) : (j == 1 ? (a & 3) >= 2 : a >= 4);
}

__host__ __device__ inline int h8_tiles(const Geometry& g) {
  return ((g.nnx + kBX - 1) / kBX) * ((g.nny + kBY - 1) / kBY) * ((g.nnz + kBZ - 1) / kBZ);
}

// tr[A] += the products of neighbour M's values u with the K0 entries that
// couple corner A to the neighbour's corner (when the neighbour is a corner
// of the element in which the node is corner A); every index and sign is a
// compile-time constant
template <int M, int A, int IC>
__device__ __forceinline__ void h8_term(double (&tr)[8][3], const double (&u)[3], const H8Row& K) {
  constexpr int mx = M % 3 - 1, my = (M / 3) % 3 - 1, mz = M / 9 - 1;
  constexpr int bx = corner_bit(A, 0) + mx, by = corner_bit(A, 1) + my, bz = corner_bit(A, 2) + mz;
  if constexpr (bx >= 0 && bx <= 1 && by >= 0 && by <= 1 && bz >= 0 && bz <= 1) {
    constexpr int I = IC / 3, C = IC % 3;
    constexpr H8Cls k = h8_class(mx != 0, my != 0, mz != 0, I, C);
    constexpr int sg = k.s * (corner_bit(A, C) ? -1 : 1);
    tr[A][I] += (sg > 0 ? K.q[k.q] : -K.q[k.q]) * u[C];
  }
}

template <int M, int A, int... IC>
__device__ __forceinline__ void h8_corner(double (&tr)[8][3], const double (&u)[3], const H8Row& K,
                                          std::integer_sequence<int, IC...>) {
  (h8_term<M, A, IC>(tr, u, K), ...);
}

template <int M, int... A>
__device__ __forceinline__ void h8_neighbour(double (&tr)[8][3], const double* __restrict__ x0,
                                             const double* __restrict__ x1,
                                             const double* __restrict__ x2, const H8Row& K,
                                             std::integer_sequence<int, A...>) {
  constexpr int off = (M % 3 - 1) + kGX * ((M / 3) % 3 - 1) + kGX * kGY * (M / 9 - 1);
  const double u[3] = {x0[off], x1[off], x2[off]};
  (h8_corner<M, A>(tr, u, K, std::make_integer_sequence<int, 9>{}), ...);
  // a row of three neighbours at a time: the next row's loads are not
  // hoisted above this row's products (fewer live registers)
  if constexpr (M % 3 == 2) __builtin_amdgcn_sched_barrier(0);
}

template <int... M>
__device__ __forceinline__ void h8_rows(double (&tr)[8][3], const double* __restrict__ x0,
                                        const double* __restrict__ x1,
                                        const double* __restrict__ x2, const H8Row& K,
                                        std::integer_sequence<int, M...>) {
  (h8_neighbour<M>(tr, x0, x1, x2, K, std::make_integer_sequence<int, 8>{}), ...);
}

// P3 and DIR as for Q4
template <bool P3, bool DIR>
__global__ __launch_bounds__(kThreads) void k_apply_h8(
    Geometry g, const double* __restrict__ rho, const double* __restrict__ x,
    double* __restrict__ y, const uint8_t* __restrict__ fixed, H8Row K, double E0, double Emin,
    double penal, double* __restrict__ parts, Gate gate, const double* __restrict__ zdir,
    double* __restrict__ pnew, const double* __restrict__ beta, int first) {
  constexpr int kGQ = (kGV + kThreads - 1) / kThreads;   // staged values per thread
  constexpr int kFQ = (kFN + kThreads - 1) / kThreads;
  __shared__ double xh[3][kGN];
  __shared__ double Eh[kFN];
  __shared__ double sh[4];
  const int sys = blockIdx.y;
  if (!gate_running(gate, sys)) return;
  const int nnx = g.nnx, nny = g.nny, nnz = g.nnz;
  const int ntx = (nnx + kBX - 1) / kBX, nty = (nny + kBY - 1) / kBY;
  const int ntiles = h8_tiles(g);
  // XCD-aware order (workgroups whose index agrees mod 8 share an XCD): each
  // such group takes a contiguous range of slots and each slot a contiguous
  // range of tiles, so that neighbouring tiles' shared halo lines meet in one L2
  const int W = gridDim.x, grp = blockIdx.x % 8, per = W / 8, rem = W % 8;
  const int slot = (grp < rem ? grp * (per + 1) : rem * (per + 1) + (grp - rem) * per) +
                   blockIdx.x / 8;
  const int tbeg = (int)((int64_t)slot * ntiles / W);
  const int tend = (int)((int64_t)(slot + 1) * ntiles / W);
  const double* xs = x + (size_t)sys * g.ndof;
  double* ys = y + (size_t)sys * g.ndof;
  const double* rs = rho + (size_t)sys * g.nel;
  const double* zs = DIR ? zdir + (size_t)sys * g.ndof : nullptr;
  double* ps = DIR ? pnew + (size_t)sys * g.ndof : nullptr;
  const double bt = DIR && !first ? beta[sys] : 0.0;
  const int t = threadIdx.x;
  const int lx = t % kBX, ly = (t / kBX) % kBY, lz = t / (kBX * kBY);
  const int hc = (lx + 1) + kGX * ((ly + 1) + kGY * (lz + 1));   // the node in the halo
  const int ec = lx + kFX * (ly + kFY * lz);   // its element at offset (-1, -1, -1)
  double acc = 0.0;
  for (int tile = tbeg; tile < tend; ++tile) {
    const int x0 = (tile % ntx) * kBX, y0 = ((tile / ntx) % nty) * kBY, z0 = tile / (ntx * nty) * kBZ;
    // the staging indices below depend on the thread only; recomputed per
    // tile (an empty asm hides that from the compiler) they hold no registers
    // through the products
    int tq = t;
    asm volatile("" : "+v"(tq));
    // every load of the tile is issued before any is used; halo rows (one per
    // (y, z) of the halo) are 3 kGX contiguous values
    double hv[kGQ];
    uint8_t hf[kGQ];
    double rv[kFQ];
#pragma unroll
    for (int q = 0; q < kGQ; ++q) {
      const int i = tq + q * kThreads;
      const int row = i / (3 * kGX), off = i - row * (3 * kGX);
      const int X = x0 - 1 + off / 3, Y = y0 - 1 + row % kGY, Z = z0 - 1 + row / kGY;
      hv[q] = 0.0;
      hf[q] = 1;
      if (i < kGV && X >= 0 && X < nnx && Y >= 0 && Y < nny && Z >= 0 && Z < nnz) {
        const int64_t dof = 3 * ((int64_t)(x0 - 1) + nnx * (Y + (int64_t)nny * Z)) + off;
        if (DIR) {
          const double zv = zs[dof];
          const double pv = first ? 0.0 : xs[dof];
          hv[q] = zv + bt * pv;
        } else {
          hv[q] = xs[dof];
        }
        hf[q] = fixed[dof];
      }
    }
#pragma unroll
    for (int q = 0; q < kFQ; ++q) {
      const int i = tq + q * kThreads;
      const int ex = x0 - 1 + i % kFX, ey = y0 - 1 + (i / kFX) % kFY, ez = z0 - 1 + i / (kFX * kFY);
      rv[q] = -1.0;   // outside the mesh
      if (i < kFN && ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely && ez >= 0 && ez < g.nelz)
        rv[q] = rs[ex + (int64_t)g.nelx * (ey + (int64_t)g.nely * ez)];
    }
    __syncthreads();   // the previous tile's LDS reads are done
#pragma unroll
    for (int q = 0; q < kGQ; ++q) {
      const int i = tq + q * kThreads;
      const int row = i / (3 * kGX), off = i - row * (3 * kGX);
      if (i < kGV) xh[off % 3][off / 3 + kGX * row] = hf[q] ? 0.0 : hv[q];
    }
#pragma unroll
    for (int q = 0; q < kFQ; ++q) {
      const int i = tq + q * kThreads;
      const double r = rv[q];
      const double E = r < 0.0 ? 0.0
                               : (P3 ? Emin + (E0 - Emin) * (r * r * r)
                                     : simp_modulus(r, E0, Emin, penal));
      if (i < kFN) Eh[i] = E;
    }
    __syncthreads();
    double tr[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) tr[a][0] = tr[a][1] = tr[a][2] = 0.0;
    h8_rows(tr, &xh[0][hc], &xh[1][hc], &xh[2][hc], K, std::make_integer_sequence<int, 27>{});
    double yv[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int cx = corner_bit(a, 0), cy = corner_bit(a, 1), cz = corner_bit(a, 2);
      const double E = Eh[ec + (1 - cx) + kFX * ((1 - cy) + kFY * (1 - cz))];
#pragma unroll
      for (int i = 0; i < 3; ++i) yv[i] += (corner_bit(a, i) ? -E : E) * tr[a][i];
    }
    const int X = x0 + lx, Y = y0 + ly, Z = z0 + lz;
    if (X < nnx && Y < nny && Z < nnz) {
      const int64_t n = X + nnx * (Y + (int64_t)nny * Z);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double pv = xh[i][hc];   // P x at the node
        const double yi = fixed[3 * n + i] ? 0.0 : yv[i];
        ys[3 * n + i] = yi;
        if (DIR) ps[3 * n + i] = pv;   // the new p
        if (parts) acc += pv * yi;
      }
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

bool h8_structured(const double* K0, double* q) {
  double mx = 0.0;
  for (int i = 0; i < 576; ++i) mx = std::max(mx, std::fabs(K0[i]));
  // each class's value from a corner-0 entry of sign +1
  bool seen[12] = {};
  for (int e = 0; e < 8; ++e)
    for (int i = 0; i < 3; ++i)
      for (int c = 0; c < 3; ++c) {
        const H8Cls k = h8_class(corner_bit(e, 0), corner_bit(e, 1), corner_bit(e, 2), i, c);
        if (k.s > 0 && !seen[k.q]) {
          q[k.q] = K0[i * 24 + 3 * e + c];
          seen[k.q] = true;
        }
      }
  for (int j = 0; j < 12; ++j)
    if (!seen[j]) return false;
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) {
          const int ex = corner_bit(a, 0) ^ corner_bit(b, 0), ey = corner_bit(a, 1) ^ corner_bit(b, 1),
                    ez = corner_bit(a, 2) ^ corner_bit(b, 2);
          const H8Cls k = h8_class(ex, ey, ez, i, c);
          const int sg = k.s * (corner_bit(a, i) ? -1 : 1) * (corner_bit(a, c) ? -1 : 1);
          if (std::fabs(K0[(3 * a + i) * 24 + 3 * b + c] - sg * q[k.q]) > 1e-14 * mx) return false;
        }
  return true;
}

int apply_parts(const Geometry& g) {
  if (g.dim == 2) return std::min(q4_tiles(g), kMaxParts);
  return std::min(h8_tiles(g), kMaxParts);
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
    H8Row q;
    std::copy(h.K0h8, h.K0h8 + 12, q.q);
#define TPCG_H8(P3, DIR)                                                                      \
  hipLaunchKernelGGL((k_apply_h8<P3, DIR>), grid, dim3(kThreads), 0, st, g, rho, x, y, h.fixed, \
                     q, pr.E0, pr.Emin, pr.penal, parts, gate, z, pnew, beta, first)
    if (z) {
      if (pr.penal == 3.0) TPCG_H8(true, true);
      else TPCG_H8(false, true);
    } else {
      if (pr.penal == 3.0) TPCG_H8(true, false);
      else TPCG_H8(false, false);
    }
#undef TPCG_H8
  }
}

}  // namespace tpcg
