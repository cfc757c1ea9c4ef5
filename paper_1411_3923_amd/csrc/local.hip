// Exact subdomain solves of the additive Schwarz preconditioner (Sec. 2.4.2:
// the local parts R_j^T A_j^-1 R_j r, A_j the principal submatrix of the
// supported stiffness matrix on the subdomain's closed-cell DOFs), one
// workgroup per (system, subdomain).
//
// A_j is factored in twisted form (btri.h): A_j = M M^T with M_bb = L_bb,
// M_{b,b-1} = A_{b,b-1} D_{b-1}^T above the middle block mid = nblk / 2 and
// M_{b,b+1} = A_{b,b+1} D_{b+1}^T below it (D_b = L_bb^-1). A record holds
// only C_b = D_b^T D_b, the inverse of the block's Schur complement; the
// off-diagonal blocks are never stored, since A_{b,b+-1} is the stiffness of
// one element layer, applied matrix-free from its moduli and the element
// matrix K0 (Sec. 2.2). With s_b = D_b^T y_b both triangular solves need one
// symmetric product per block, and they run from the two ends towards the
// middle and back, as two chains of half the length:
//   M y = r    s_b = C_b (r_b - A_{b,b-1} s_{b-1}),   b = 0 .. mid - 1
//              s_b = C_b (r_b - A_{b,b+1} s_{b+1}),   b = nblk - 1 .. mid + 1
//   M^T x = y  x_mid = C_mid (r_mid - A_{mid,mid-1} s_{mid-1} - A_{mid,mid+1} s_{mid+1})
//              x_b = s_b - C_b A_{b,b+1} x_{b+1},    b = mid - 1 .. 0
//              x_b = s_b - C_b A_{b,b-1} x_{b-1},    b = mid + 1 .. nblk - 1
// (s and x enter the couplings with supported DOFs zeroed.)
//
// The two chains advance in lockstep and share the barriers: per block one
// phase for the product (thread tau holds tile tau of both chains' current
// records in registers and writes its partial products), one for the row
// sums (the thread owning a row adds its partials in a fixed order) and one
// for the couplings into the next block. The next record is requested as
// soon as the product is formed, and the barriers order LDS traffic only,
// so the load flies across the two other phases.
#include "big.h"
#include "btri.h"

namespace tpcg {

namespace {

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

__host__ __device__ inline int strip_width(const Geometry& g) {
  return g.dim == 3 ? (g.bn + 1) * (g.bn + 1) : g.bn + 1;
}

// LDS in elements of T: K0 [nd][nd]; per chain the tile partials [nt][np]
// and the vectors a, c [np]; the two exchanged vectors [np] (the lower
// chain's coupling into block mid, and x_mid); the element-layer moduli
// [nblk - 1][sw]; then nloc bytes of support flags.
__host__ __device__ inline size_t chain_lds_elems(const Geometry& g) {
  const TileShape ts = tile_shape(g.nb);
  return (size_t)ts.nt * 4 * ts.nt + 2 * (size_t)4 * ts.nt;
}
__host__ __device__ inline size_t local_elems(const Geometry& g) {
  return (size_t)g.ndpe * g.ndpe + 2 * chain_lds_elems(g) + 8 * (size_t)tile_shape(g.nb).nt +
         (size_t)(g.nblk - 1) * strip_width(g);
}

size_t local_solve_lds_bytes(const Geometry& g, size_t elem) {
  return ((local_elems(g) * elem + 15) & ~(size_t)15) + (((size_t)g.nloc + 15) & ~(size_t)15);
}

// Steps K = 0 .. 2 mid: the upper chain (c = 0) runs blocks 0 .. mid - 1
// (forward), mid (K = mid), mid - 1 .. 0 (backward); the lower chain (c = 1)
// runs blocks nblk - 1 .. mid + 1 (K < nbot) and mid + 1 .. nblk - 1
// (K = mid + 1 ..) and idles otherwise. Thread tau < nl holds tile tau (and
// tau + 256 when TPT = 2) of both chains' records; DOF o of chain c's node
// layer belongs to thread 128 c + o. zloc receives s and then x, in box
// order.
template <typename T, int TPT, int D>
__global__ __launch_bounds__(kThreads) void k_local_solves(
    Geometry g, const double* __restrict__ r, const T* __restrict__ lfac,
    const T* __restrict__ emod, const uint8_t* __restrict__ fixed, const double* __restrict__ K0,
    T* __restrict__ zloc, int nchains, Gate gate) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int CH = 2;
  const int id = blockIdx.x;
  if (id >= nchains) return;
  const int sys = id / g.nsub, j = id - (id / g.nsub) * g.nsub;
  if (!gate_running(gate, sys)) return;   // uniform over the workgroup

  constexpr int d = D, nd = D == 3 ? 24 : 8;
  const int nb = g.nb, nblk = g.nblk, bn = g.bn;
  const TileShape ts = tile_shape(nb);
  const int nt = ts.nt, np = 4 * ts.nt, nl = ts.nl;
  const int sw = strip_width(g);
  const int mid = nblk / 2, nbot = nblk - 1 - mid;
  const int t = threadIdx.x;
  // the row phases of the two chains run on different waves
  int o[CH];
  bool ow[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    o[c] = t - c * (kThreads / CH);
    ow[c] = o[c] >= 0 && o[c] < nb;
  }
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  const double* rs = r + (size_t)sys * g.ndof;
  const T* es = emod + (size_t)sys * g.nel;
  T* zs = zloc + (size_t)id * g.nloc;
  const T* F = lfac + (size_t)id * nblk * ts.tstride;

  const size_t cl = chain_lds_elems(g);
  T* K0s = reinterpret_cast<T*>(smem);
  T* red[CH];   // [nt][np] tile partials
  T* va[CH];    // t_b (forward) / w_b (backward)
  T* vc[CH];    // masked s_b (forward) / masked x_b (backward)
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    red[c] = K0s + nd * nd + c * cl;
    va[c] = red[c] + (size_t)nt * np;
    vc[c] = va[c] + np;
  }
  T* cm = K0s + nd * nd + CH * cl;   // A_{mid,mid+1} s_{mid+1} from the lower chain
  T* xm = cm + np;                   // masked x_mid for the lower chain
  T* strip = xm + np;                // moduli of element layer L at strip + L sw
  uint8_t* fx = smem + ((local_elems(g) * sizeof(T) + 15) & ~(size_t)15);

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
    const V* src = reinterpret_cast<const V*>(F + (size_t)b * ts.tstride);
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
  // y = C x for the symmetric C from its lower tiles, as partial products in
  // disjoint slots: tile (I, J) writes (C_IJ x_J) to red[J][4I + i] and, off
  // the diagonal, (C_IJ^T x_I) to red[I][4J + k]; row o is then the sum of
  // red[K][o] over all K (K <= o / 4 from the tiles left of the diagonal,
  // K > o / 4 from those below it)
  auto prod_sym = [&](int c, const T* x) {
#pragma unroll
    for (int u = 0; u < TPT; ++u)
      if (tau[u] < nl) {
        const T* xj = x + 4 * tJ[u];
        const T* xi = x + 4 * tI[u];
        const T j0 = xj[0], j1 = xj[1], j2 = xj[2], j3 = xj[3];
        const T i0 = xi[0], i1 = xi[1], i2 = xi[2], i3 = xi[3];
        T* on = red[c] + (size_t)tJ[u] * np + 4 * tI[u];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          on[i] = tl[c][u][4 * i] * j0 + tl[c][u][4 * i + 1] * j1 + tl[c][u][4 * i + 2] * j2 +
                  tl[c][u][4 * i + 3] * j3;
        if (tI[u] != tJ[u]) {
          T* ot = red[c] + (size_t)tI[u] * np + 4 * tJ[u];
#pragma unroll
          for (int k = 0; k < 4; ++k)
            ot[k] = tl[c][u][k] * i0 + tl[c][u][4 + k] * i1 + tl[c][u][8 + k] * i2 +
                    tl[c][u][12 + k] * i3;
        }
      }
  };
  // row o's partials, added in order K = 0 .. nt - 1 (unrolled by four, so
  // that four reads are in flight ahead of their sums)
  auto row_sum = [&](int c, int oo) {
    T s = 0;
#pragma unroll 4
    for (int K = 0; K < nt; ++K) s += red[c][(size_t)K * np + oo];
    return s;
  };
  // the box DOFs of chain c's row in block b: one stride per block (a node
  // row in 2-d, a node layer in 3-d) from the row's DOF in block 0
  const int64_t lstride = (int64_t)d * g.nnx * (d == 3 ? g.nny : 1);
  int64_t dof0[CH];
  int lxo[CH], lyo[CH], co[CH];   // the row's node in the layer and its component
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int oc = ow[c] ? o[c] : 0;
    dof0[c] = box_dof(g, jx, jy, jz, oc);
    const int m = oc / d;
    co[c] = oc - m * d;
    lxo[c] = m % bn;
    lyo[c] = d == 3 ? m / bn : 0;
  }
  auto rhs = [&](int c, int b) { return (T)rs[dof0[c] + b * lstride]; };
  auto coupling = [&](int c, int L, const T* v, bool top) {
    return layer_coupling_at<D>(bn, K0s, strip + (size_t)L * sw, v, lxo[c], lyo[c], co[c], top);
  };

  // set-up: first records, K0, layer moduli, support flags, zeroed vectors,
  // first right-hand sides
  const bool lower_runs = nbot > 0;
  T rn[CH], yb[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    rn[c] = 0;
    yb[c] = 0;
    if (c == 0 || lower_runs) load_tiles(c, c == 0 ? 0 : nblk - 1);
  }
  for (int i = t; i < nd * nd; i += kThreads) K0s[i] = (T)K0[i];
  for (int i = t; i < (nblk - 1) * sw; i += kThreads) {
    const int L = i / sw, q = i - (i / sw) * sw;
    const int qx = q % (bn + 1), qy = q / (bn + 1);
    const int ex = g.s * jx - 1 + qx;
    const int ey = d == 3 ? g.s * jy - 1 + qy : g.s * jy + L;
    const int ez = d == 3 ? g.s * jz + L : 0;
    const bool in = ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely;
    strip[i] = in ? es[ex + (int64_t)g.nelx * (ey + (int64_t)g.nely * ez)] : (T)0;
  }
  for (int l = t; l < g.nloc; l += kThreads) fx[l] = fixed[box_dof(g, jx, jy, jz, l)];
#pragma unroll
  for (int c = 0; c < CH; ++c)
    for (int i = t; i < 2 * np; i += kThreads) va[c][i] = 0;   // va, vc
  for (int i = t; i < 2 * np; i += kThreads) cm[i] = 0;        // cm, xm
  lds_barrier();
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    if (!ow[c] || (c == 1 && !lower_runs)) continue;
    const int b0 = c == 0 ? 0 : nblk - 1, b1 = c == 0 ? 1 : nblk - 2;
    va[c][o[c]] = rhs(c, b0);                 // t_b0 = r_b0
    if (c == 0 ? b1 <= mid : b1 >= mid + 1) rn[c] = rhs(c, b1);
  }

  for (int K = 0; K <= 2 * mid; ++K) {
    lds_barrier();
    if (K == mid && lower_runs) {
      // t_mid -= A_{mid,mid+1} s_{mid+1}, from the lower chain
      if (ow[0] && !fx[mid * nb + o[0]]) va[0][o[0]] -= cm[o[0]];
      lds_barrier();
    }
    if (K == mid + 1 && lower_runs) {
      // lower chain: w_{mid+1} = A_{mid+1,mid} x_mid, s_{mid+1} from the forward pass
      if (ow[1]) {
        va[1][o[1]] = fx[(mid + 1) * nb + o[1]] ? (T)0 : coupling(1, mid, xm, true);
        yb[1] = zs[(mid + 1) * nb + o[1]];
      }
      lds_barrier();
    }
    // activity and block of each chain at this step
    bool act[CH], fwd[CH], middle[CH];
    int b[CH];
    act[0] = true;
    fwd[0] = K < mid;
    middle[0] = K == mid;
    b[0] = K <= mid ? K : 2 * mid - K;
    fwd[1] = K < nbot;
    middle[1] = false;
    b[1] = fwd[1] ? nblk - 1 - K : K;
    act[1] = fwd[1] || (K >= mid + 1 && K <= mid + nbot);

#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (!act[c]) continue;
      prod_sym(c, va[c]);                        // C_b t_b  or  C_b w_b
      // the record has served its block: request the next one (the lower
      // chain keeps its block mid + 1 from its last forward step to its
      // first backward one)
      int nx;
      if (c == 0) nx = K < mid ? K + 1 : b[c] - 1;
      else if (fwd[c]) nx = b[c] - 1 >= mid + 1 ? b[c] - 1 : -1;
      else nx = b[c] + 1 < nblk ? b[c] + 1 : -1;
      if (nx >= 0) load_tiles(c, nx);
    }
    lds_barrier();
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (!act[c] || !ow[c]) continue;
      const T sum = row_sum(c, o[c]);
      // forward: s_b; middle: x_mid; backward: x_b = s_b - C_b w_b
      const T val = (fwd[c] || middle[c]) ? sum : yb[c] - sum;
      zs[b[c] * nb + o[c]] = val;
      const T sm = fx[b[c] * nb + o[c]] ? (T)0 : val;
      vc[c][o[c]] = sm;
      if (middle[c]) xm[o[c]] = sm;
    }
    lds_barrier();
    // couplings into the next step of each chain
    if (act[0] && ow[0]) {
      const int bc = b[0];
      if (fwd[0]) {
        // t_{b+1} = r_{b+1} - A_{b+1,b} s_b
        va[0][o[0]] = fx[(bc + 1) * nb + o[0]] ? rn[0] : rn[0] - coupling(0, bc, vc[0], true);
        if (bc + 2 <= mid) rn[0] = rhs(0, bc + 2);
      } else if (bc >= 1) {
        // w_{b-1} = A_{b-1,b} x_b, and s_{b-1} back from the forward pass
        va[0][o[0]] = fx[(bc - 1) * nb + o[0]] ? (T)0 : coupling(0, bc - 1, vc[0], false);
        yb[0] = zs[(bc - 1) * nb + o[0]];
      }
    }
    if (act[1] && ow[1]) {
      const int bc = b[1];
      if (fwd[1] && bc == mid + 1) {
        cm[o[1]] = coupling(1, mid, vc[1], false);   // A_{mid,mid+1} s_{mid+1}
      } else if (fwd[1]) {
        // t_{b-1} = r_{b-1} - A_{b-1,b} s_b
        va[1][o[1]] = fx[(bc - 1) * nb + o[1]] ? rn[1] : rn[1] - coupling(1, bc - 1, vc[1], false);
        if (bc - 2 >= mid + 1) rn[1] = rhs(1, bc - 2);
      } else if (bc + 1 < nblk) {
        // w_{b+1} = A_{b+1,b} x_b, and s_{b+1} back from the forward pass
        va[1][o[1]] = fx[(bc + 1) * nb + o[1]] ? (T)0 : coupling(1, bc, vc[1], true);
        yb[1] = zs[(bc + 1) * nb + o[1]];
      }
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

template <typename T, int TPT, int D>
void local_launch_as(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  const int nchains = nsys * g.nsub;
  static bool done = false;
  allow_lds(&k_local_solves<T, TPT, D>, done);
  hipLaunchKernelGGL((k_local_solves<T, TPT, D>), dim3(nchains), dim3(kThreads),
                     local_solve_lds_bytes(g, sizeof(T)), st, g, r,
                     reinterpret_cast<const T*>(h.lfac), reinterpret_cast<const T*>(h.emod),
                     h.fixed, h.K0, reinterpret_cast<T*>(h.zloc), nchains, gate);
}

template <typename T>
void local_launch(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st) {
  // one tile per thread where it suffices
  const bool one = tile_shape(h.g.nb).nl <= kThreads;
  if (h.g.dim == 2) {
    if (one) local_launch_as<T, 1, 2>(h, r, nsys, gate, st);
    else local_launch_as<T, 2, 2>(h, r, nsys, gate, st);
  } else {
    if (one) local_launch_as<T, 1, 3>(h, r, nsys, gate, st);
    else local_launch_as<T, 2, 3>(h, r, nsys, gate, st);
  }
}

}  // namespace

void launch_local_solves(Handle& h, const double* r, int nsys, const Gate& gate,
                         hipStream_t st) {
  if (h.big) {
    if (h.mixed)
      big_local_solves<float>(h.g, r, reinterpret_cast<const float*>(h.lfac),
                              reinterpret_cast<const float*>(h.emod), h.fixed, h.K0,
                              reinterpret_cast<float*>(h.zloc), nsys, gate, st);
    else
      big_local_solves<double>(h.g, r, reinterpret_cast<const double*>(h.lfac),
                               reinterpret_cast<const double*>(h.emod), h.fixed, h.K0,
                               reinterpret_cast<double*>(h.zloc), nsys, gate, st);
    return;
  }
  if (h.mixed) local_launch<float>(h, r, nsys, gate, st);
  else local_launch<double>(h, r, nsys, gate, st);
}

}  // namespace tpcg
