// Exact subdomain solves of the additive Schwarz preconditioner (Sec. 2.4.2:
// the local parts R_j^T A_j^-1 R_j r, A_j the principal submatrix of the
// supported stiffness matrix on the subdomain's closed-cell DOFs), one
// workgroup per (system, subdomain).
//
// The factor of A_j is kept as the tiled inverted diagonal blocks D_b of its
// block-tridiagonal Cholesky factor (btri.h); the off-diagonal factor blocks
// are never stored: B_{b+1} = A_{b+1,b} D_b^T, and A_{b+1,b} is applied
// matrix-free from the moduli of the element layer between node layers b and
// b + 1 and the element matrix K0 (Sec. 2.2). Per block the workgroup forms
// D_b v and D_b^T v from register tiles, 4 x 4 per thread, with the partial
// sums of each row combined in LDS by the thread owning that row, in a fixed
// order. Each record is requested as soon as the previous one has been used
// for both products of its block; the other workgroups on the compute unit
// cover the latency.
#include "btri.h"

namespace tpcg {

namespace {

// (A_{b+1,b} v)[o] for a DOF o of node layer b + 1 (top = true, v on layer b)
// or (A_{b+1,b}^T v)[o] for a DOF o of layer b (top = false, v on layer
// b + 1): the stiffness of the element layer between the two node layers,
// E[] its moduli indexed (ex + 1) + (bn + 1) (ey + 1) over box-local element
// coordinates, zero outside the mesh. Supported DOFs are masked by the caller.
template <typename T>
__device__ inline T layer_coupling(int d, int bn, const T* __restrict__ K0s,
                                   const T* __restrict__ E, const T* __restrict__ v, int o,
                                   bool top) {
  const int nd = d == 3 ? 24 : 8;
  const int m = o / d, c = o - m * d;
  const int lx = m % bn, ly = d == 3 ? m / bn : 0;
  const int ny = d == 3 ? 2 : 1, ylim = d == 3 ? bn : 1;
  T acc = 0;
  for (int hy = 0; hy < ny; ++hy)
    for (int hx = 0; hx < 2; ++hx) {
      // element with this node at its corner (hx, hy) of the top or bottom face
      const int ex = lx - hx, ey = ly - hy;
      const T Ee = E[(ex + 1) + (d == 3 ? (bn + 1) * (ey + 1) : 0)];
      const int ca = d == 3 ? corner_of(hx, hy, top) : corner_of(hx, top, 0);
      T s = 0;
      for (int oy = 0; oy < ny; ++oy)
        for (int ox = 0; ox < 2; ++ox) {
          const int px = ex + ox, py = ey + oy;
          if (px < 0 || px >= bn || py < 0 || py >= ylim) continue;
          const int cb = d == 3 ? corner_of(ox, oy, !top) : corner_of(ox, !top, 0);
          const T* kr = K0s + (d * ca + c) * nd + d * cb;
          const T* vp = v + d * (px + bn * py);
          for (int c2 = 0; c2 < d; ++c2) s += kr[c2] * vp[c2];
        }
      acc += Ee * s;
    }
  return acc;
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};

// LDS elements (of T) of k_local_solves; nloc bytes of support flags follow
size_t local_solve_lds_elems(const Geometry& g) {
  const TileShape ts = tile_shape(g.nb);
  const int np = 4 * ts.nt;
  const int sw = g.dim == 3 ? (g.bn + 1) * (g.bn + 1) : g.bn + 1;
  return (size_t)ts.nt * np + 3 * (size_t)np + (size_t)g.ndpe * g.ndpe +
         (size_t)(g.nblk - 1) * sw;
}

// Thread tau < nl holds tile tau (and tau + 256 when TPT = 2) of the current
// record; thread o < nb owns DOF o of the current node layer. The block steps
// run 0, 1, ..., nblk - 1 (forward, the last one also giving x_{nblk-1}) and
// then nblk - 2, ..., 0 (backward). zloc receives the forward intermediate y
// and then the solution, in box order.
template <typename T, int TPT>
__global__ __launch_bounds__(kThreads) void k_local_solves(
    Geometry g, const double* __restrict__ r, const T* __restrict__ lfac,
    const T* __restrict__ emod, const uint8_t* __restrict__ fixed, const double* __restrict__ K0,
    T* __restrict__ zloc, Gate gate) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int sys = blockIdx.x / g.nsub;
  const int j = blockIdx.x - sys * g.nsub;
  if (!gate_running(gate, sys)) return;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  const int d = g.dim, nb = g.nb, nblk = g.nblk, bn = g.bn, nd = g.ndpe;
  const TileShape ts = tile_shape(nb);
  const int nt = ts.nt, np = 4 * nt, nl = ts.nl;
  const int sw = d == 3 ? (bn + 1) * (bn + 1) : bn + 1;
  T* red = reinterpret_cast<T*>(smem);          // [nt][np] tile partials
  T* va = red + (size_t)nt * np;                // t_b (forward) / w_b (backward)
  T* vb = va + np;                              // y_b (forward) / v_b (backward)
  T* vc = vb + np;                              // masked s_b (forward) / masked x_{b+1} (backward)
  T* K0s = vc + np;
  T* strip = K0s + nd * nd;                     // [nblk - 1][sw] element-layer moduli
  uint8_t* fx = reinterpret_cast<uint8_t*>(strip + (size_t)(nblk - 1) * sw);
  const int t = threadIdx.x;
  const bool own = t < nb;
  const double* rs = r + (size_t)sys * g.ndof;
  const T* es = emod + (size_t)sys * g.nel;
  T* zs = zloc + ((size_t)sys * g.nsub + j) * g.nloc;
  const T* F = lfac + ((size_t)sys * g.nsub + j) * nblk * ts.tstride;

  typedef typename Vec16<T>::type V;
  typedef T Tiles[TPT][16];
  constexpr int per = 16 / (int)sizeof(T);
  constexpr int nvl = 16 / per;
  int tI[TPT], tJ[TPT], tau[TPT];
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    tau[u] = t + kThreads * u;
    tI[u] = 0;
    tJ[u] = 0;
    if (tau[u] < nl) tile_rc(tau[u], tI[u], tJ[u]);
  }
  auto load_tiles = [&](Tiles& tl, int b) {
    const V* src = reinterpret_cast<const V*>(F + (size_t)b * ts.tstride);
#pragma unroll
    for (int u = 0; u < TPT; ++u)
      if (tau[u] < nl) {
#pragma unroll
        for (int v = 0; v < nvl; ++v) {
          const V q = src[(size_t)v * nl + tau[u]];
#pragma unroll
          for (int w = 0; w < per; ++w) tl[u][v * per + w] = q[w];
        }
      }
  };
  // red[J][4I + i] = (D_IJ x_J)[i]
  auto prod_n = [&](const Tiles& tl, const T* x) {
#pragma unroll
    for (int u = 0; u < TPT; ++u)
      if (tau[u] < nl) {
        const T* xv = x + 4 * tJ[u];
        const T x0 = xv[0], x1 = xv[1], x2 = xv[2], x3 = xv[3];
        T* o = red + (size_t)tJ[u] * np + 4 * tI[u];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          o[i] = tl[u][4 * i] * x0 + tl[u][4 * i + 1] * x1 + tl[u][4 * i + 2] * x2 +
                 tl[u][4 * i + 3] * x3;
      }
  };
  // red[I][4J + c] = (D_IJ^T x_I)[c]
  auto prod_t = [&](const Tiles& tl, const T* x) {
#pragma unroll
    for (int u = 0; u < TPT; ++u)
      if (tau[u] < nl) {
        const T* xv = x + 4 * tI[u];
        const T x0 = xv[0], x1 = xv[1], x2 = xv[2], x3 = xv[3];
        T* o = red + (size_t)tI[u] * np + 4 * tJ[u];
#pragma unroll
        for (int c = 0; c < 4; ++c)
          o[c] = tl[u][c] * x0 + tl[u][4 + c] * x1 + tl[u][8 + c] * x2 + tl[u][12 + c] * x3;
      }
  };
  auto sum_n = [&](int o) {
    T s = 0;
    for (int J = 0; J <= o / 4; ++J) s += red[(size_t)J * np + o];
    return s;
  };
  auto sum_t = [&](int o) {
    T s = 0;
    for (int I = o / 4; I < nt; ++I) s += red[(size_t)I * np + o];
    return s;
  };
  auto rhs = [&](int b) { return (T)rs[box_dof(g, jx, jy, jz, b * nb + t)]; };

  const int nsteps = 2 * nblk - 1;
  T rn = 0, yb = 0;
  Tiles tl;
  auto step = [&](int k) {
    if (k < nblk) {
      // forward: y_b = D_b t_b, s_b = D_b^T y_b, t_{b+1} = r_{b+1} - A_{b+1,b} s_b
      const int b = k;
      prod_n(tl, va);
      __syncthreads();
      if (own) {
        const T y = sum_n(t);
        vb[t] = y;
        zs[b * nb + t] = y;
      }
      __syncthreads();
      prod_t(tl, vb);                            // for the last block this is x_{nblk-1}
      // the record has been used twice: request the next one
      if (k + 1 < nsteps) load_tiles(tl, k + 1 < nblk ? k + 1 : 2 * nblk - 3 - k);
      __syncthreads();
      if (own) {
        const T s = sum_t(t);
        vc[t] = fx[b * nb + t] ? (T)0 : s;
        if (b + 1 == nblk) zs[b * nb + t] = s;
      }
      __syncthreads();
      if (b + 1 < nblk) {
        if (own) {
          const bool f = fx[(b + 1) * nb + t];
          va[t] = f ? rn : rn - layer_coupling(d, bn, K0s, strip + (size_t)b * sw, vc, t, true);
          if (b + 2 < nblk) rn = rhs(b + 2);
        }
        __syncthreads();
      } else if (own && nblk > 1) {
        yb = zs[(nblk - 2) * nb + t];
      }
    } else {
      // backward: w_b = A_{b+1,b}^T x_{b+1}, v_b = y_b - D_b w_b, x_b = D_b^T v_b
      const int b = 2 * nblk - 2 - k;
      if (own)
        va[t] = fx[b * nb + t] ? (T)0
                               : layer_coupling(d, bn, K0s, strip + (size_t)b * sw, vc, t, false);
      __syncthreads();
      prod_n(tl, va);
      __syncthreads();
      if (own) {
        vb[t] = yb - sum_n(t);
        if (b >= 1) yb = zs[(b - 1) * nb + t];
      }
      __syncthreads();
      prod_t(tl, vb);
      if (k + 1 < nsteps) load_tiles(tl, 2 * nblk - 3 - k);
      __syncthreads();
      if (own) {
        const T x = sum_t(t);
        zs[b * nb + t] = x;
        vc[t] = fx[b * nb + t] ? (T)0 : x;
      }
      __syncthreads();
    }
  };

  // set-up: first record, K0, layer moduli, support flags, zeroed padding
  if (own) rn = rhs(0);
  load_tiles(tl, 0);
  for (int i = t; i < nd * nd; i += kThreads) K0s[i] = (T)K0[i];
  for (int i = t; i < (nblk - 1) * sw; i += kThreads) {
    const int b = i / sw, q = i - (i / sw) * sw;
    const int qx = q % (bn + 1), qy = q / (bn + 1);
    const int ex = g.s * jx - 1 + qx;
    const int ey = d == 3 ? g.s * jy - 1 + qy : g.s * jy + b;
    const int ez = d == 3 ? g.s * jz + b : 0;
    const bool in = ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely;
    strip[i] = in ? es[ex + (int64_t)g.nelx * (ey + (int64_t)g.nely * ez)] : (T)0;
  }
  for (int l = t; l < g.nloc; l += kThreads) fx[l] = fixed[box_dof(g, jx, jy, jz, l)];
  for (int i = t; i < 3 * np; i += kThreads) va[i] = 0;
  __syncthreads();
  if (own) va[t] = rn;                           // t_0 = r_0
  if (own && nblk > 1) rn = rhs(1);
  __syncthreads();
  for (int k = 0; k < nsteps; ++k) step(k);
}

template <typename K>
void allow_lds(K kernel, bool& done) {
  if (done) return;
  hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();   // an unsupported size must not leave a stale error behind
  done = true;
}

template <typename T>
void local_launch(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  const size_t lds = sizeof(T) * local_solve_lds_elems(g) + (size_t)g.nloc;
  const T* fac = reinterpret_cast<const T*>(h.lfac);
  const T* em = reinterpret_cast<const T*>(h.emod);
  T* zl = reinterpret_cast<T*>(h.zloc);
  const dim3 grid(nsys * g.nsub);
  if (tile_shape(g.nb).nl <= kThreads) {
    static bool done = false;
    allow_lds(&k_local_solves<T, 1>, done);
    hipLaunchKernelGGL((k_local_solves<T, 1>), grid, dim3(kThreads), lds, st, g, r, fac, em,
                       h.fixed, h.K0, zl, gate);
  } else {
    static bool done = false;
    allow_lds(&k_local_solves<T, 2>, done);
    hipLaunchKernelGGL((k_local_solves<T, 2>), grid, dim3(kThreads), lds, st, g, r, fac, em,
                       h.fixed, h.K0, zl, gate);
  }
}

}  // namespace

void launch_local_solves(Handle& h, const double* r, int nsys, const Gate& gate,
                         hipStream_t st) {
  if (h.mixed) local_launch<float>(h, r, nsys, gate, st);
  else local_launch<double>(h, r, nsys, gate, st);
}

}  // namespace tpcg
