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

// LDS of one chain in elements of T: tile partials [nt][np], three vectors of
// np, the element-layer moduli [nblk - 1][sw]; nloc bytes of support flags
// per chain follow all chains, K0 precedes them.
__host__ __device__ inline size_t chain_lds_elems(const Geometry& g) {
  const TileShape ts = tile_shape(g.nb);
  const int np = 4 * ts.nt;
  const int sw = g.dim == 3 ? (g.bn + 1) * (g.bn + 1) : g.bn + 1;
  return (size_t)ts.nt * np + 3 * (size_t)np + (size_t)(g.nblk - 1) * sw;
}

size_t local_solve_lds_bytes(const Geometry& g, int ch, size_t elem) {
  return elem * ((size_t)g.ndpe * g.ndpe + ch * chain_lds_elems(g)) +
         ch * (((size_t)g.nloc + 15) & ~(size_t)15);
}

// CH independent chains (system, subdomain) per workgroup, advanced in
// lockstep so that they share the barriers and keep CH records in flight.
// Thread tau < nl holds tile tau (and tau + 256 when TPT = 2) of each chain's
// current record; thread o < nb owns DOF o of each chain's current node
// layer. The block steps run 0, 1, ..., nblk - 1 (forward, the last one also
// giving x_{nblk-1}) and then nblk - 2, ..., 0 (backward). zloc receives the
// forward intermediate y and then the solution, in box order.
template <typename T, int TPT, int CH>
__global__ __launch_bounds__(kThreads) void k_local_solves(
    Geometry g, const double* __restrict__ r, const T* __restrict__ lfac,
    const T* __restrict__ emod, const uint8_t* __restrict__ fixed, const double* __restrict__ K0,
    T* __restrict__ zloc, int nchains, Gate gate) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int d = g.dim, nb = g.nb, nblk = g.nblk, bn = g.bn, nd = g.ndpe;
  const TileShape ts = tile_shape(nb);
  const int nt = ts.nt, np = 4 * ts.nt, nl = ts.nl;
  const int sw = d == 3 ? (bn + 1) * (bn + 1) : bn + 1;
  const int t = threadIdx.x;
  // DOF o of chain c's node layer belongs to thread c * (kThreads / CH) + o,
  // so the chains' row phases run on different waves
  int o[CH];
  bool ow[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    o[c] = t - c * (kThreads / CH);
    ow[c] = o[c] >= 0 && o[c] < nb;
  }

  // chains of this workgroup; a chain whose system has stopped only follows
  // the barriers
  bool run[CH];
  int jx[CH], jy[CH], jz[CH];
  const double* rs[CH];
  const T* es[CH];
  const T* F[CH];
  T* zs[CH];
  bool any = false;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int id = blockIdx.x * CH + c;
    const int sys = id / g.nsub, j = id - (id / g.nsub) * g.nsub;
    run[c] = id < nchains && gate_running(gate, sys);
    any |= run[c];
    sub_coords(g, j, jx[c], jy[c], jz[c]);
    rs[c] = r + (size_t)sys * g.ndof;
    es[c] = emod + (size_t)sys * g.nel;
    zs[c] = zloc + (size_t)id * g.nloc;
    F[c] = lfac + (size_t)id * nblk * ts.tstride;
  }
  if (!any) return;

  const size_t cl = chain_lds_elems(g);
  T* K0s = reinterpret_cast<T*>(smem);
  T* red[CH];   // [nt][np] tile partials
  T* va[CH];   // t_b (forward) / w_b (backward)
  T* vb[CH];   // y_b (forward) / v_b (backward)
  T* vc[CH];   // masked s_b (forward) / masked x_{b+1} (backward)
  T* strip[CH];
  uint8_t* fx[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    red[c] = K0s + nd * nd + c * cl;
    va[c] = red[c] + (size_t)nt * np;
    vb[c] = va[c] + np;
    vc[c] = vb[c] + np;
    strip[c] = vc[c] + np;
    fx[c] = reinterpret_cast<uint8_t*>(K0s + nd * nd + CH * cl) +
            c * (((size_t)g.nloc + 15) & ~(size_t)15);
  }

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
  Tiles tl[CH];
  auto load_tiles = [&](int c, int b) {
    const V* src = reinterpret_cast<const V*>(F[c] + (size_t)b * ts.tstride);
#pragma unroll
    for (int u = 0; u < TPT; ++u)
      if (tau[u] < nl) {
#pragma unroll
        for (int v = 0; v < nvl; ++v) {
          const V q = src[(size_t)v * nl + tau[u]];
#pragma unroll
          for (int w = 0; w < per; ++w) tl[c][u][v * per + w] = q[w];
        }
      }
  };
  // red[J][4I + i] = (D_IJ x_J)[i]
  auto prod_n = [&](int c, const T* x) {
#pragma unroll
    for (int u = 0; u < TPT; ++u)
      if (tau[u] < nl) {
        const T* xv = x + 4 * tJ[u];
        const T x0 = xv[0], x1 = xv[1], x2 = xv[2], x3 = xv[3];
        T* o = red[c] + (size_t)tJ[u] * np + 4 * tI[u];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          o[i] = tl[c][u][4 * i] * x0 + tl[c][u][4 * i + 1] * x1 + tl[c][u][4 * i + 2] * x2 +
                 tl[c][u][4 * i + 3] * x3;
      }
  };
  // red[I][4J + k] = (D_IJ^T x_I)[k]
  auto prod_t = [&](int c, const T* x) {
#pragma unroll
    for (int u = 0; u < TPT; ++u)
      if (tau[u] < nl) {
        const T* xv = x + 4 * tI[u];
        const T x0 = xv[0], x1 = xv[1], x2 = xv[2], x3 = xv[3];
        T* o = red[c] + (size_t)tI[u] * np + 4 * tJ[u];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          o[k] = tl[c][u][k] * x0 + tl[c][u][4 + k] * x1 + tl[c][u][8 + k] * x2 +
                 tl[c][u][12 + k] * x3;
      }
  };
  auto sum_n = [&](int c, int o) {
    T s = 0;
    for (int J = 0; J <= o / 4; ++J) s += red[c][(size_t)J * np + o];
    return s;
  };
  auto sum_t = [&](int c, int o) {
    T s = 0;
    for (int I = o / 4; I < nt; ++I) s += red[c][(size_t)I * np + o];
    return s;
  };
  auto rhs = [&](int c, int b) {
    return (T)rs[c][box_dof(g, jx[c], jy[c], jz[c], b * nb + o[c])];
  };

  // set-up: first records, K0, layer moduli, support flags, zeroed padding
  T rn[CH], yb[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    rn[c] = 0;
    yb[c] = 0;
    if (run[c]) {
      if (ow[c]) rn[c] = rhs(c, 0);
      load_tiles(c, 0);
    }
  }
  for (int i = t; i < nd * nd; i += kThreads) K0s[i] = (T)K0[i];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    if (!run[c]) continue;
    for (int i = t; i < (nblk - 1) * sw; i += kThreads) {
      const int b = i / sw, q = i - (i / sw) * sw;
      const int qx = q % (bn + 1), qy = q / (bn + 1);
      const int ex = g.s * jx[c] - 1 + qx;
      const int ey = d == 3 ? g.s * jy[c] - 1 + qy : g.s * jy[c] + b;
      const int ez = d == 3 ? g.s * jz[c] + b : 0;
      const bool in = ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely;
      strip[c][i] = in ? es[c][ex + (int64_t)g.nelx * (ey + (int64_t)g.nely * ez)] : (T)0;
    }
    for (int l = t; l < g.nloc; l += kThreads) fx[c][l] = fixed[box_dof(g, jx[c], jy[c], jz[c], l)];
    for (int i = t; i < 3 * np; i += kThreads) va[c][i] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    if (!run[c] || !ow[c]) continue;
    va[c][o[c]] = rn[c];                            // t_0 = r_0
    if (nblk > 1) rn[c] = rhs(c, 1);
  }
  __syncthreads();

  // Block steps k = 0 .. nsteps - 1: forward block b = k, then backward
  // block b = 2 nblk - 2 - k. Entering a step, va holds t_b (forward) or
  // w_b = A_{b+1,b}^T x_{b+1} (backward) and tl holds D_b.
  const int nsteps = 2 * nblk - 1;
  for (int k = 0; k < nsteps; ++k) {
    const bool fwd = k < nblk;
    const int b = fwd ? k : 2 * nblk - 2 - k;
#pragma unroll
    for (int c = 0; c < CH; ++c)
      if (run[c]) prod_n(c, va[c]);              // D_b t_b  or  D_b w_b
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (!run[c] || !ow[c]) continue;
      const T sn = sum_n(c, o[c]);
      if (fwd) {
        vb[c][o[c]] = sn;                           // y_b
        zs[c][b * nb + o[c]] = sn;
      } else {
        vb[c][o[c]] = yb[c] - sn;                   // v_b = y_b - D_b w_b
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (!run[c]) continue;
      prod_t(c, vb[c]);                          // s_b = D_b^T y_b  or  x_b = D_b^T v_b
      // the record has been used twice: request the next one
      if (k + 1 < nsteps) load_tiles(c, k + 1 < nblk ? k + 1 : 2 * nblk - 3 - k);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (!run[c] || !ow[c]) continue;
      const T st = sum_t(c, o[c]);
      vc[c][o[c]] = fx[c][b * nb + o[c]] ? (T)0 : st;
      if (!fwd || b + 1 == nblk) zs[c][b * nb + o[c]] = st;   // x_b (x_{nblk-1} = s_{nblk-1})
    }
    __syncthreads();
    if (k + 1 < nsteps) {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        if (!run[c] || !ow[c]) continue;
        if (k + 1 < nblk) {
          // t_{b+1} = r_{b+1} - A_{b+1,b} s_b
          const bool f = fx[c][(b + 1) * nb + o[c]];
          va[c][o[c]] = f ? rn[c]
                       : rn[c] - layer_coupling(d, bn, K0s, strip[c] + (size_t)b * sw, vc[c],
                                                o[c], true);
          if (b + 2 < nblk) rn[c] = rhs(c, b + 2);
        } else {
          // w_e = A_{e+1,e}^T x_{e+1} for the next backward block e
          const int e = 2 * nblk - 3 - k;
          va[c][o[c]] = fx[c][e * nb + o[c]]
                         ? (T)0
                         : layer_coupling(d, bn, K0s, strip[c] + (size_t)e * sw, vc[c], o[c], false);
          yb[c] = zs[c][e * nb + o[c]];             // y_e from the forward pass
        }
      }
      __syncthreads();
    }
  }
}

template <typename K>
void allow_lds(K kernel, bool& done) {
  if (done) return;
  hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();   // an unsupported size must not leave a stale error behind
  done = true;
}

template <typename T, int TPT, int CH>
void local_launch_as(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  const int nchains = nsys * g.nsub;
  static bool done = false;
  allow_lds(&k_local_solves<T, TPT, CH>, done);
  hipLaunchKernelGGL((k_local_solves<T, TPT, CH>), dim3((nchains + CH - 1) / CH), dim3(kThreads),
                     local_solve_lds_bytes(g, CH, sizeof(T)), st, g, r,
                     reinterpret_cast<const T*>(h.lfac), reinterpret_cast<const T*>(h.emod),
                     h.fixed, h.K0, reinterpret_cast<T*>(h.zloc), nchains, gate);
}

template <typename T>
void local_launch(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st) {
  // two chains per workgroup where one tile per thread suffices
  if (tile_shape(h.g.nb).nl <= kThreads) local_launch_as<T, 1, 2>(h, r, nsys, gate, st);
  else local_launch_as<T, 2, 1>(h, r, nsys, gate, st);
}

}  // namespace

void launch_local_solves(Handle& h, const double* r, int nsys, const Gate& gate,
                         hipStream_t st) {
  if (h.mixed) local_launch<float>(h, r, nsys, gate, st);
  else local_launch<double>(h, r, nsys, gate, st);
}

}  // namespace tpcg
