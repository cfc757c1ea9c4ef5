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

// LDS elements (of T) of k_local_solves, plus nloc bytes of support flags
__host__ __device__ inline size_t local_solve_lds_elems(const Geometry& g) {
  const TileShape ts = tile_shape(g.nb);
  const int np = 4 * ts.nt;
  const int sw = g.dim == 3 ? (g.bn + 1) * (g.bn + 1) : g.bn + 1;
  return (size_t)ts.nt * np + 3 * (size_t)np + (size_t)g.ndpe * g.ndpe +
         (size_t)(g.nblk - 1) * sw;
}

// Exact subdomain solves z_j = A_j^-1 R_j r, one workgroup per (system,
// subdomain), with the tiled D_b records and the matrix-free layer coupling
// (see btri.h). Thread tau < nl holds tile tau of the current record in
// registers (TPT tiles per thread when nl > 256); thread o < nb owns DOF o of
// the current node layer. Per block, D_b v and D_b^T v are formed as tile
// partials in LDS and summed by the owning threads in a fixed order. The next
// record is requested as soon as the current one has been used twice.
// Results (and the forward-pass intermediate y) go to zloc in box order.
template <typename T, int TPT>
__global__ __launch_bounds__(kThreads) void k_local_solves(
    Geometry g, const double* __restrict__ r, const T* __restrict__ lfac,
    const T* __restrict__ emod, const uint8_t* __restrict__ fixed, const double* __restrict__ K0,
    T* __restrict__ zloc, Gate gate) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sh[4];
  const int sys = blockIdx.x / g.nsub;
  const int j = blockIdx.x - sys * g.nsub;
  if (!gate_running(gate, sys, sh)) return;
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
  constexpr int per = 16 / (int)sizeof(T);
  constexpr int nvl = 16 / per;
  int tI[TPT], tJ[TPT], tau[TPT];
  T tl[TPT][16];
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    tau[u] = t + kThreads * u;
    tI[u] = 0;
    tJ[u] = 0;
    if (tau[u] < nl) tile_rc(tau[u], tI[u], tJ[u]);
  }
  auto load_tiles = [&](int b) {
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
  auto prod_n = [&](const T* x) {
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
  auto prod_t = [&](const T* x) {
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

  // set-up: K0, layer moduli, support flags, zeroed vector padding
  T rn = own ? rhs(0) : (T)0;
  load_tiles(0);
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

  // forward: y_b = D_b t_b, s_b = D_b^T y_b, t_{b+1} = r_{b+1} - A_{b+1,b} s_b
  for (int b = 0; b < nblk; ++b) {
    prod_n(va);
    __syncthreads();
    if (own) {
      const T y = sum_n(t);
      vb[t] = y;
      zs[b * nb + t] = y;
    }
    __syncthreads();
    prod_t(vb);                                  // for the last block this is x_{nblk-1}
    if (b + 1 < nblk) load_tiles(b + 1);
    else if (nblk > 1) load_tiles(nblk - 2);
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
    }
  }
  // backward: w_b = A_{b+1,b}^T x_{b+1}, v_b = y_b - D_b w_b, x_b = D_b^T v_b
  T yb = (own && nblk > 1) ? zs[(nblk - 2) * nb + t] : (T)0;
  for (int b = nblk - 2; b >= 0; --b) {
    if (own)
      va[t] = fx[b * nb + t] ? (T)0
                             : layer_coupling(d, bn, K0s, strip + (size_t)b * sw, vc, t, false);
    __syncthreads();
    prod_n(va);
    __syncthreads();
    if (own) {
      vb[t] = yb - sum_n(t);
      if (b >= 1) yb = zs[(b - 1) * nb + t];
    }
    __syncthreads();
    prod_t(vb);
    if (b >= 1) load_tiles(b - 1);
    __syncthreads();
    if (own) {
      const T x = sum_t(t);
      zs[b * nb + t] = x;
      vc[t] = fx[b * nb + t] ? (T)0 : x;
    }
    __syncthreads();
  }
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

template <typename T>
void local_launch(Handle& h, const double* r, int nsys, const Gate& gate, hipStream_t st) {
  const Geometry& g = h.g;
  const size_t lds = sizeof(T) * local_solve_lds_elems(g) + (size_t)g.nloc;
  const T* fac = reinterpret_cast<const T*>(h.lfac);
  const T* em = reinterpret_cast<const T*>(h.emod);
  T* zl = reinterpret_cast<T*>(h.zloc);
  if (tile_shape(g.nb).nl <= kThreads) {
    static bool done = false;
    set_lds_once(&k_local_solves<T, 1>, done);
    hipLaunchKernelGGL((k_local_solves<T, 1>), dim3(nsys * g.nsub), dim3(kThreads), lds, st, g,
                       r, fac, em, h.fixed, h.K0, zl, gate);
  } else {
    static bool done = false;
    set_lds_once(&k_local_solves<T, 2>, done);
    hipLaunchKernelGGL((k_local_solves<T, 2>), dim3(nsys * g.nsub), dim3(kThreads), lds, st, g,
                       r, fac, em, h.fixed, h.K0, zl, gate);
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
