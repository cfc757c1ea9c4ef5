// Batched block-tridiagonal Cholesky factorisation into the packed or the
// tiled record format of btri.h (one workgroup per matrix), the
// multi-right-hand-side solve used by the subspace iteration of the local
// eigenproblems, and the dense inverse of a packed factor.
//
// The O(nb^3) work runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
// Lane layout of the instruction: A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k, result D[i][j] in lane j + 16 (i % 4), register i / 4. Per block row:
//   A_bb -= B_b B_b^T                         16 x 16 tiles on MFMA
//   A_bb = L_bb L_bb^T                        16-column panels: the panel in
//                                             registers (readlane broadcasts),
//                                             trailing tiles on MFMA
//   D_b = L_bb^-1 in place                    diagonal tiles by substitution in
//                                             registers, off-diagonal tiles
//                                             D_IJ = -D_II sum_K L_IK D_KJ on MFMA,
//                                             one tile column per wave
//   B_{b+1} = A_{b+1,b} D_b^T in place        MFMA, each wave owns its row tiles
// Rows and columns past nb read as zero. Two nb x nb LDS buffers suffice, so
// blocks of up to 96 fit.
#include "btri.h"

namespace tpcg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline double lget(const double* M, int ld, int nb, int r, int c) {
  return (r < nb && c < nb) ? M[r * ld + c] : 0.0;
}

// acc += A[ra.., k] * Bm[rb.., k]^T over k in [k0, k1) (k0 multiple of 4).
// The operands of four k-steps are read from clamped addresses before their
// MFMAs and masked after one wait (the empty asm keeps the compiler from
// moving each read under its bounds test, which would serialise them).
__device__ inline d4 mfma_nt(const double* A, const double* Bm, int ld, int nb, int ra, int rb,
                             int k0, int k1, d4 acc) {
  const int l = threadIdx.x & 63;
  const int li = l & 15, lk = l >> 4;
  const int a_off = min(ra + li, nb - 1) * ld, b_off = min(rb + li, nb - 1) * ld;
  const bool a_in = ra + li < nb, b_in = rb + li < nb;
  int k = k0;
  for (; k + 16 <= k1; k += 16) {
    double a[4], b[4];
    bool ka[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = k + 4 * u + lk, cc = min(c, nb - 1);
      ka[u] = c < nb;
      a[u] = A[a_off + cc];
      b[u] = Bm[b_off + cc];
    }
    asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(b[0]), "+v"(b[1]),
                 "+v"(b[2]), "+v"(b[3]));
#pragma unroll
    for (int u = 0; u < 4; ++u)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a_in && ka[u] ? a[u] : 0.0,
                                                b_in && ka[u] ? b[u] : 0.0, acc, 0, 0, 0);
  }
  for (; k < k1; k += 4) {
    const int c = k + lk, cc = min(c, nb - 1);
    double a = A[a_off + cc], b = Bm[b_off + cc];
    asm volatile("" : "+v"(a), "+v"(b));
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a_in && c < nb ? a : 0.0, b_in && c < nb ? b : 0.0,
                                              acc, 0, 0, 0);
  }
  return acc;
}


// orders the LDS traffic of one wave
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int kMaxTiles = (kMaxNb + 15) / 16;

// LDS (doubles) of the stencil input: two element layers of moduli, K0, the
// Neumann diagonals of two node layers and the support flags of the three
// node layers those element layers touch
__host__ __device__ inline int layer_width(const Geometry& g) {
  return g.dim == 3 ? (g.bn + 1) * (g.bn + 1) : g.bn + 1;
}
__host__ __device__ inline size_t stencil_lds_elems(const Geometry& g) {
  return 2 * (size_t)layer_width(g) + (size_t)g.ndpe * g.ndpe + 2 * (size_t)g.nb +
         (3 * (size_t)g.nb + 7) / 8;
}

// Box-local coordinates of local DOF l: x, y (3D), layer (the block axis), component.
struct BoxNode {
  int x, y, lay, c;
};
__device__ inline BoxNode box_node(const Geometry& g, int l) {
  const int ln = l / g.dim;
  BoxNode n;
  n.c = l - ln * g.dim;
  n.x = ln % g.bn;
  if (g.dim == 3) {
    n.y = (ln / g.bn) % g.bn;
    n.lay = ln / (g.bn * g.bn);
  } else {
    n.y = 0;
    n.lay = ln / g.bn;
  }
  return n;
}

// Moduli of element layers L0 and L0 + 1 (layer L lies between node layers L
// and L + 1; -1 and nblk - 1 are outside the box) into Es, zero outside the
// mesh and, for the Neumann matrices, outside the cell; the support flags of
// node layers L0, L0 + 1, L0 + 2 into fl. PRE: the moduli are read from
// em (the system's block of si.emod) instead of being formed from the
// densities.
template <bool PRE = false>
__device__ void stage_layers(const StencilIn& si, int jx, int jy, int jz, int L0, double* Es,
                             uint8_t* fl, int tid = threadIdx.x, const double* em = nullptr) {
  const Geometry& g = si.g;
  const int d = g.dim, ew = layer_width(g), s = g.s;
  for (int i = tid; i < 3 * g.nb; i += kThreads) {
    const int L = L0 + i / g.nb;
    fl[i] = (L >= 0 && L < g.nblk) ? si.fixed[box_dof(g, jx, jy, jz, L * g.nb + i % g.nb)] : 0;
  }
  for (int i = tid; i < 2 * ew; i += kThreads) {
    const int L = L0 + i / ew, q = i - (i / ew) * ew;
    const int qx = q % (g.bn + 1), qy = q / (g.bn + 1);
    const int ex = s * jx - 1 + qx;
    const int ey = d == 3 ? s * jy - 1 + qy : s * jy + L;
    const int ez = d == 3 ? s * jz + L : 0;
    bool in = ex >= 0 && ex < g.nelx && ey >= 0 && ey < g.nely && ez >= 0 && ez < g.nelz;
    if (si.neumann)
      in = in && ex >= s * jx && ex < s * jx + s && ey >= s * jy && ey < s * jy + s &&
           (d == 2 || (ez >= s * jz && ez < s * jz + s));
    const int64_t el = ex + (int64_t)g.nelx * (ey + (int64_t)g.nely * ez);
    if (PRE)
      Es[i] = in ? em[el] : 0.0;
    else
      Es[i] = in ? simp_modulus(si.rho[el], si.E0, si.Emin, si.penal) : 0.0;
  }
}

// Stiffness entry K(lr, lc) over the staged element layers (the node layers
// of lr and lc differ by at most one and are covered by L0, L0 + 1).
__device__ double stencil_entry(const Geometry& g, int lr, int lc, int L0, const double* Es,
                                const double* K0s) {
  const BoxNode a = box_node(g, lr), b = box_node(g, lc);
  if (abs(a.x - b.x) > 1 || abs(a.y - b.y) > 1 || abs(a.lay - b.lay) > 1) return 0.0;
  const int d = g.dim, nd = g.ndpe, ew = layer_width(g);
  const int y0 = d == 3 ? max(a.y, b.y) - 1 : 0, y1 = d == 3 ? min(a.y, b.y) : 0;
  double v = 0.0;
  for (int L = max(a.lay, b.lay) - 1; L <= min(a.lay, b.lay); ++L)
    for (int ey = y0; ey <= y1; ++ey)
      for (int ex = max(a.x, b.x) - 1; ex <= min(a.x, b.x); ++ex) {
        const double E = Es[(L - L0) * ew + (ex + 1) + (d == 3 ? (g.bn + 1) * (ey + 1) : 0)];
        const int ar = d == 3 ? corner_of(a.x - ex, a.y - ey, a.lay - L)
                              : corner_of(a.x - ex, a.lay - L, 0);
        const int ac = d == 3 ? corner_of(b.x - ex, b.y - ey, b.lay - L)
                              : corner_of(b.x - ex, b.lay - L, 0);
        v += E * K0s[(d * ar + a.c) * nd + d * ac + b.c];
      }
  return v;
}

// One workgroup per matrix. Input: assembled blocks A[b][0] = A_bb,
// A[b][1] = A_{b,b-1} (FP64, row-major nb x nb), or, when si.rho is set, the
// subdomain stiffness matrix of subdomain blockIdx.x computed block by block
// from the element moduli (the Dirichlet matrix, or the scaled shifted
// Neumann matrix with D^-1/2 written to si.dis). Output: packed or tiled
// records in T. flag[0] = 1 on a non-positive pivot (replaced by 1 so that
// the factorisation completes and the caller can report it).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_btri_factor(const double* __restrict__ A,
                                                         T* __restrict__ out, BtriShape sh,
                                                         int* __restrict__ flag, int tiles,
                                                         StencilIn si) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nb = sh.nb, nblk = sh.nblk, pe = sh.pe;
  const int ld = lds_ld(nb);
  const int NT = (nb + 15) / 16;
  double* X = reinterpret_cast<double*>(smem);   // A_bb -> L_bb -> D_b
  double* Y = X + (size_t)nb * ld;                // B_b, then A_{b+1,b} -> B_{b+1}
  double* tmp = Y + (size_t)nb * ld;              // 16 x 16 per wave
  const size_t msz = (size_t)nb * nb;
  const double* F = A + (size_t)blockIdx.x * nblk * 2 * msz;
  const TileShape tsh = tile_shape(nb);
  const int rstride = tiles ? tsh.tstride : sh.bstride;
  T* O = out + (size_t)blockIdx.x * nblk * rstride;
  const int t = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63;   // wave index, uniform
  const int li = l & 15, lq = l >> 4;
  double* tw = tmp + wv * 256;
  // stencil input: staged moduli, K0 and the Neumann diagonals of the last
  // two node layers (by parity)
  const bool sten = si.rho != nullptr;
  double* Es = tmp + 4 * 256;
  double* K0s = Es + 2 * (sten ? layer_width(si.g) : 0);
  double* dl = K0s + (sten ? si.g.ndpe * si.g.ndpe : 0);
  uint8_t* fl = reinterpret_cast<uint8_t*>(dl + (sten ? 2 * nb : 0));   // flags of 3 node layers
  int jx = 0, jy = 0, jz = 0;
  if (sten) {
    sub_coords(si.g, phys_sub(si.g, blockIdx.x), jx, jy, jz);
    for (int i = t; i < si.g.ndpe * si.g.ndpe; i += kThreads) K0s[i] = si.K0[i];
  }
  // Neumann diagonal of node layer L (needs the layers L - 1 and L staged
  // at L0), D^-1/2 to si.dis
  auto diag_layer = [&](int L, int L0) {
    for (int i = t; i < nb; i += kThreads) {
      const int lr = L * nb + i;
      const bool fx = fl[(L - L0) * nb + i];
      const double dd = stencil_entry(si.g, lr, lr, L0, Es, K0s);
      dl[(L & 1) * nb + i] = dd;
      if (si.dis) si.dis[(size_t)blockIdx.x * si.g.nloc + lr] = fx ? 0.0 : 1.0 / sqrt(dd);
    }
  };
  // block (Lr, Lc) of the subdomain matrix from the staged layers
  // Entries whose in-layer indices lie further apart than any two
  // neighbouring nodes' DOFs (2d - 1 in 2d, d(bn + 1) + d - 1 in 3d) are
  // structural zeros and skip the node decoding and the stencil.
  const int span = sten ? (si.g.dim == 3 ? si.g.dim * (si.g.bn + 2) - 1 : 2 * si.g.dim - 1) : 0;
  auto fill = [&](double* dst, int Lr, int Lc, int L0) {
    for (int r = t / 16; r < nb; r += kThreads / 16)
      for (int c = t % 16; c < nb; c += 16) {
        const int lr = Lr * nb + r, lc = Lc * nb + c;
        double v = 0.0;
        if (abs(r - c) <= span) {
          if (fl[(Lr - L0) * nb + r] || fl[(Lc - L0) * nb + c]) {
            v = lr == lc ? (si.neumann ? si.fixed_diag + si.shift : 1.0) : 0.0;
          } else {
            v = stencil_entry(si.g, lr, lc, L0, Es, K0s);
            if (si.neumann)
              v = v / sqrt(dl[(Lr & 1) * nb + r] * dl[(Lc & 1) * nb + c]) +
                  (lr == lc ? si.shift : 0.0);
          }
        }
        dst[r * ld + c] = v;
      }
  };
  auto load = [&](double* dst, const double* src) {
    // one flat, unrolled sweep: several loads of each thread in flight at once
    const int n2 = nb * nb;
#pragma unroll 8
    for (int e = t; e < n2; e += kThreads) {
      const int r = e / nb;
      dst[r * ld + e - r * nb] = src[e];
    }
  };
  // Twisted order (stencil input with si.twist set): the node layers below
  // the middle block mid = nblk / 2 are eliminated upwards from the last one
  // (blocks nblk - 1, ..., mid + 1, records at their own index), their Schur
  // term for block mid is parked in si.twist, then the layers 0, ..., mid
  // are eliminated downwards and block mid receives both terms.
  const bool twist = sten && si.twist != nullptr;
  const int mid = nblk / 2;
  const int nbot = twist ? nblk - 1 - mid : 0;
  double* TS = twist ? si.twist + (size_t)blockIdx.x * ((size_t)nb * (nb + 1) / 2) : nullptr;
  if (sten) {
    // block B needs the element layers B - 1 and B
    const int b0 = nbot > 0 ? nblk - 1 : 0;
    stage_layers(si, jx, jy, jz, b0 - 1, Es, fl);
    __syncthreads();
    if (si.neumann) diag_layer(0, -1);
    __syncthreads();
    fill(X, b0, b0, b0 - 1);
  } else {
    load(X, F);
  }
  for (int step = 0; step < nblk; ++step) {
    const bool bot = step < nbot;
    const int b = bot ? nblk - 1 - step : step - nbot;
    __syncthreads();
    if (step != 0 && step != nbot) {
      // A_bb -= B_b B_b^T on the lower tiles
      int tile = 0;
      for (int I = 0; I < NT; ++I)
        for (int J = 0; J <= I; ++J, ++tile) {
          if ((tile & 3) != wv) continue;
          d4 acc = {0.0, 0.0, 0.0, 0.0};
          acc = mfma_nt(Y, Y, ld, nb, 16 * I, 16 * J, 0, (nb + 3) & ~3, acc);
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * I + 4 * v + lq, c = 16 * J + li;
            if (r < nb && c < nb) X[r * ld + c] -= acc[v];
          }
        }
      __syncthreads();
    }
    if (nbot > 0 && !bot && b == mid) {
      // the middle block also takes the Schur term of the lower half
      for (int e = t; e < nb * nb; e += kThreads) {
        const int r = e / nb, c = e - (e / nb) * nb;
        if (c <= r) X[r * ld + c] += TS[(size_t)r * (r + 1) / 2 + c];
      }
      __syncthreads();
    }
    // blocked Cholesky: panel p (16 columns) in the registers of wave 0,
    // then the trailing tiles on MFMA
    for (int p = 0; p < NT; ++p) {
      const int c0 = 16 * p, c1 = min(nb, c0 + 16);
      if (wv == 0) {
        const int w = c1 - c0;
        double x[2][16];   // lane l holds panel rows c0 + l and c0 + l + 64
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int r = c0 + l + 64 * s;
#pragma unroll
          for (int cc = 0; cc < 16; ++cc) x[s][cc] = (r < nb && cc < w) ? X[r * ld + c0 + cc] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c < w) {
            double piv = bcast_lane(x[0][c], c);      // row c0 + c lives in lane c
            if (!(piv > 0.0)) {
              if (l == 0) flag[0] = 1;
              piv = 1.0;
            }
            const double dcc = sqrt(piv);
            const double inv = 1.0 / dcc;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
              const int rr = l + 64 * s;
              if (rr == c) x[s][c] = dcc;
              else if (rr > c) x[s][c] *= inv;
            }
#pragma unroll
            for (int cc = c + 1; cc < 16; ++cc) {
              if (cc < w) {
                const double lcc = bcast_lane(x[0][c], cc);
#pragma unroll
                for (int s = 0; s < 2; ++s)
                  if (l + 64 * s >= cc) x[s][cc] -= x[s][c] * lcc;
              }
            }
          }
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int r = c0 + l + 64 * s;
#pragma unroll
          for (int cc = 0; cc < 16; ++cc)
            if (r < nb && cc < w) X[r * ld + c0 + cc] = x[s][cc];
        }
      }
      __syncthreads();
      int tile = 0;
      for (int I = p + 1; I < NT; ++I)
        for (int J = p + 1; J <= I; ++J, ++tile) {
          if ((tile & 3) != wv) continue;
          d4 acc = {0.0, 0.0, 0.0, 0.0};
          acc = mfma_nt(X, X, ld, nb, 16 * I, 16 * J, c0, c0 + 16, acc);
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * I + 4 * v + lq, c = 16 * J + li;
            if (r < nb && c < nb) X[r * ld + c] -= acc[v];
          }
        }
      __syncthreads();
    }
    // D = L^-1 in place. Diagonal tiles first: lane li of a wave solves
    // L_II y = e_li in registers (all its reads precede its writes, and the
    // lanes of a wave move in lockstep)
    for (int I = wv; I < NT; I += 4) {
      if (li == l) {
        const int j = 16 * I + li;
        double y[16];
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) {
          const int r = 16 * I + ii;
          double s = (ii == li) ? 1.0 : 0.0;
#pragma unroll
          for (int c = 0; c < ii; ++c) s -= lget(X, ld, nb, r, 16 * I + c) * y[c];
          y[ii] = r < nb ? s / lget(X, ld, nb, r, r) : 0.0;
        }
        wave_sync();
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) {
          const int r = 16 * I + ii;
          if (r < nb && j < nb) X[r * ld + j] = y[ii];
        }
      }
    }
    __syncthreads();
    // off-diagonal tiles, rows top-down within a column:
    // D_IJ = -D_II sum_{K=J}^{I-1} L_IK D_KJ. The columns are independent, so
    // wave w sweeps J = w, w + 4, ...; the new tiles go to Y (free until the
    // next coupling block is loaded), which leaves in X the L tiles that the
    // other columns still read, and are copied back once all columns are done.
    for (int J = wv; J + 1 < NT; J += 4)
      for (int I = J + 1; I < NT; ++I) {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int k = 16 * J; k < 16 * I; k += 4) {
          const int kr = k + lq;   // row of D_KJ: the diagonal tile lives in X, the others in Y
          const double a = lget(X, ld, nb, 16 * I + li, kr);
          const double bb = kr < 16 * J + 16 ? lget(X, ld, nb, kr, 16 * J + li)
                                             : lget(Y, ld, nb, kr, 16 * J + li);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) tw[(4 * v + lq) * 16 + li] = acc[v];
        wave_sync();
        d4 acc2 = {0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < 16; k += 4) {
          const double a = lget(X, ld, nb, 16 * I + li, 16 * I + k + lq);
          const double bb = tw[(k + lq) * 16 + li];
          acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc2, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * I + 4 * v + lq, c = 16 * J + li;
          if (r < nb && c < nb) Y[r * ld + c] = -acc2[v];
        }
        wave_sync();
      }
    __syncthreads();
    for (int e = t; e < nb * nb; e += kThreads) {
      const int r = e / nb, c = e - (e / nb) * nb;
      if ((r >> 4) > (c >> 4)) X[r * ld + c] = Y[r * ld + c];
    }
    __syncthreads();
    const bool last = step + 1 == nblk;
    const bool last_bot = bot && step + 1 == nbot;
    // next block row nr and the staged element layers L0, L0 + 1: downwards
    // (b, b + 1) serve A_{b+1,b} now and A_{b+1,b+1} below; upwards
    // (b - 2, b - 1) serve A_{b-1,b} and A_{b-1,b-1}
    const int nr = bot ? (last_bot ? mid : b - 1) : b + 1;
    const int L0 = bot ? b - 2 : b;
    if (!last) {
      // B = A_{nr,b} D^T; wave w owns row tiles I = w, w + 4, ...
      if (sten) {
        stage_layers(si, jx, jy, jz, L0, Es, fl);
        __syncthreads();
        if (si.neumann) diag_layer(b + 1, b);
        __syncthreads();
        fill(Y, nr, b, L0);
      } else {
        load(Y, F + ((size_t)(b + 1) * 2 + 1) * msz);
      }
      __syncthreads();
      for (int I = wv; I < NT; I += 4) {
        d4 acc[kMaxTiles];
#pragma unroll
        for (int J = 0; J < kMaxTiles; ++J) {
          acc[J] = d4{0.0, 0.0, 0.0, 0.0};
          if (J < NT)   // D row 16J + j is zero right of column 16J + j
            acc[J] = mfma_nt(Y, X, ld, nb, 16 * I, 16 * J, 0, min((nb + 3) & ~3, 16 * J + 16),
                             acc[J]);
        }
        wave_sync();
#pragma unroll
        for (int J = 0; J < kMaxTiles; ++J)
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * I + 4 * v + lq, c = 16 * J + li;
            if (J < NT && r < nb && c < nb) Y[r * ld + c] = acc[J][v];
          }
      }
      __syncthreads();
    }
    T* R = O + (size_t)b * rstride;
    if (tiles) {
      // record b: the lower 4 x 4 tiles of C_b = D_b^T D_b (the inverse of
      // the block's Schur complement, symmetric; its diagonal tiles in full),
      // thread-major. 16 x 16 tiles (P, Q), P >= Q, on MFMA, one per wave in
      // turn: C_PQ = sum_{K >= P} D_KP^T D_KQ over the lower triangle of D.
      {
        auto dget = [&](int r, int c) { return (r < nb && c <= r) ? X[r * ld + c] : 0.0; };
        int tile = 0;
        for (int P = 0; P < NT; ++P)
          for (int Q = 0; Q <= P; ++Q, ++tile) {
            if ((tile & 3) != wv) continue;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int k = 16 * P; k < 16 * NT; k += 4) {
              const double a = dget(k + lq, 16 * P + li);   // A[i][kk] = D[k + kk][16 P + i]
              const double bb = dget(k + lq, 16 * Q + li);  // B[kk][j] = D[k + kk][16 Q + j]
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int r = 16 * P + 4 * v + lq, c = 16 * Q + li;
              const int I = r >> 2, J = c >> 2;
              if (I < tsh.nt && J <= I)
                R[tile_offset<T>(tsh.nl, I * (I + 1) / 2 + J, 4 * (r & 3) + (c & 3))] = (T)acc[v];
            }
          }
      }
      if (!last) {
        __syncthreads();
        if (last_bot) {
          // Schur term -B B^T of the lower half for block mid, lower triangle
          int tile = 0;
          for (int I = 0; I < NT; ++I)
            for (int J = 0; J <= I; ++J, ++tile) {
              if ((tile & 3) != wv) continue;
              d4 acc = {0.0, 0.0, 0.0, 0.0};
              acc = mfma_nt(Y, Y, ld, nb, 16 * I, 16 * J, 0, (nb + 3) & ~3, acc);
              for (int v = 0; v < 4; ++v) {
                const int r = 16 * I + 4 * v + lq, c = 16 * J + li;
                if (r < nb && c <= r) TS[(size_t)r * (r + 1) / 2 + c] = -acc[v];
              }
            }
          __syncthreads();
          // then the upper half starts at block 0
          stage_layers(si, jx, jy, jz, -1, Es, fl);
          __syncthreads();
          fill(X, 0, 0, -1);
        } else if (sten) {
          fill(X, nr, nr, L0);
        } else {
          load(X, F + (size_t)(b + 1) * 2 * msz);
        }
      }
      continue;
    }
    // record b: lower(D_b) | strict upper(B_{b+1}) | band of B_{b+1}
    for (int e = t; e < nb * nb; e += kThreads) {
      const int r = e / nb, c = e - (e / nb) * nb;
      const double v = c <= r ? X[r * ld + c] : (last ? 0.0 : Y[r * ld + c]);
      R[e] = (T)v;
    }
    for (int e = t; e < nb * pe; e += kThreads) {
      const int r = e / pe, tt = e - (e / pe) * pe;
      const double v = (last || r - tt < 0) ? 0.0 : Y[r * ld + r - tt];
      R[nb * nb + e] = (T)v;
    }
    for (int e = nb * nb + nb * pe + t; e < sh.bstride; e += kThreads) R[e] = (T)0;
    if (!last) {
      __syncthreads();
      if (sten) fill(X, b + 1, b + 1, b);
      else load(X, F + (size_t)(b + 1) * 2 * msz);
    }
  }
}

// Y = (L L^T)^-1 X for every matrix, m <= kMaxSub right-hand sides, FP64,
// X and Y [nmat][n][m] row-major (n = nb * nblk).
template <int MAXV>
__global__ __launch_bounds__(kThreads) void k_btri_solve_multi(const double* __restrict__ fac,
                                                              BtriShape sh, int m,
                                                              const double* __restrict__ X,
                                                              double* __restrict__ Y) {
  extern __shared__ __align__(16) unsigned char smem[];
  const size_t n = (size_t)sh.nb * sh.nblk;
  const double* F = fac + (size_t)blockIdx.x * sh.nblk * sh.bstride;
  const double* Xj = X + (size_t)blockIdx.x * n * m;
  double* Yj = Y + (size_t)blockIdx.x * n * m;
  const int nb = sh.nb;
  btri_solve16<MAXV>(
      F, sh, m, [&](int b, int i, int r) { return Xj[((size_t)b * nb + i) * m + r]; },
      [&](int b, int i, int r) -> double& { return Yj[((size_t)b * nb + i) * m + r]; }, smem);
}

// Dense inverse of a packed factor: X = (L L^T)^-1 I, kMaxSub columns per
// workgroup; grid.x = nmat * chunks. Xinv [nmat][n][n], row-major (symmetric).
template <int MAXV>
__global__ __launch_bounds__(kThreads) void k_btri_inverse(const double* __restrict__ fac,
                                                          BtriShape sh, int chunks,
                                                          double* __restrict__ Xinv) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int mat = blockIdx.x / chunks;
  const int c0 = (blockIdx.x - mat * chunks) * kMaxSub;
  const int n = sh.nb * sh.nblk;
  const int nr = min(kMaxSub, n - c0);
  const double* F = fac + (size_t)mat * sh.nblk * sh.bstride;
  double* Xm = Xinv + (size_t)mat * n * n;
  const int nb = sh.nb;
  btri_solve16<MAXV>(
      F, sh, nr, [&](int b, int i, int r) { return (b * nb + i == c0 + r) ? 1.0 : 0.0; },
      [&](int b, int i, int r) -> double& { return Xm[(size_t)(b * nb + i) * n + c0 + r]; },
      smem, c0 / nb);
}

// ---------------------------------------------------------------------------
// Local Dirichlet factors of the subdomain solves, through the Schur
// complements of the twisted elimination (btri.h):
//   S_b = A_bb - A_{b,p} C_p A_{p,b},   C_b = S_b^-1,
// p the previous block of b's half (b - 1 above the middle block, b + 1 below
// it; none for the first block of a half), and the middle block with both
// terms. The solves need C_b only, so no Cholesky factor is formed.
//
// S_b lives in registers: thread (ti, tj) of an R x C grid owns rows
// ti + R a (a < SR) and columns tj + C q (q < SC), R = ceil(nb / SR),
// C = ceil(nb / SC); rows and columns past nb stay exactly zero throughout,
// so no access needs a bounds test. A_{b,p} and A_bb have at most 3 d
// entries per row (the nodes next to a node in a layer, all components),
// stored sparse; the correction is two sparse passes over C_p in LDS
// (T = C_p A_{p,b}, then A_{b,p} T), and A_bb is scattered into a cleared
// dense buffer. S_b is inverted in place by Gauss-Jordan elimination, which
// needs no pivoting on a symmetric positive definite matrix: step k, with
// pivot p = s_kk, maps s_ij to z_ij - c_i r_j, where z is s with column k
// replaced by the unit vector e_k, r is row k with r_k = 1, c_i = s_ik / p
// (i != k) and c_k = 1 - 1 / p. The pivot row and column go through LDS,
// double buffered so that one barrier per step suffices.
struct LfShape {
  int SR, SC;             // register block per thread
  int R, C, NR, NC, ld;   // thread grid, padded rows and columns, LDS leading dimension
};

constexpr LfShape lf_shape(int nb, int SR, int SC) {
  LfShape f{};
  f.SR = SR;
  f.SC = SC;
  f.R = (nb + SR - 1) / SR;
  f.C = (nb + SC - 1) / SC;
  f.NR = f.R * SR;
  f.NC = f.C * SC;
  f.ld = (f.NR > f.NC ? f.NR : f.NC) | 1;
  return f;
}

// the smallest register block whose thread grid fits the workgroup
constexpr LfShape lf_pick_shape(int nb) {
  constexpr int blocks[][2] = {{1, 1}, {1, 2}, {2, 2}, {2, 3}, {3, 3},
                               {3, 4}, {3, 6}, {4, 6}, {6, 6}};
  for (const auto& b : blocks) {
    const LfShape f = lf_shape(nb, b[0], b[1]);
    if (f.R * f.C <= kThreads) return f;
  }
  return LfShape{};
}

__host__ __device__ inline int coupling_nz(const Geometry& g) { return g.dim == 3 ? 27 : 6; }

__host__ __device__ inline size_t local_factor_lds_bytes(const Geometry& g, const LfShape& f) {
  const size_t np = (size_t)f.ld, nz = coupling_nz(g);
  const size_t dbl = (size_t)f.NR * f.ld + 2 * np * nz + 4 * np + 2 * (size_t)layer_width(g) +
                     (size_t)g.ndpe * g.ndpe;
  return dbl * sizeof(double) + np * nz * sizeof(int) + 3 * (size_t)g.nb;
}

// NB = g.nb: the block size is a compile-time constant, so that the
// register block, the thread grid and the LDS offsets are immediates
template <typename T, int NB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NB <= 66 ? 3 : 2))) void k_local_factor(StencilIn si, T* __restrict__ out,
                                                          int* __restrict__ flag, size_t ostride) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Geometry& g = si.g;
  constexpr LfShape f = lf_pick_shape(NB);
  constexpr int SR = f.SR, SC = f.SC, R = f.R, C = f.C, ld = f.ld, nb = NB;
  static_assert(SR > 0, "block size too large for the local factorisation");
  const int nblk = g.nblk, d = g.dim, bn = g.bn, nd = g.ndpe, nz = coupling_nz(g);
  const TileShape tsh = tile_shape(nb);
  double* Cp = reinterpret_cast<double*>(smem);   // C_p, then T, then A_bb [NR][ld]
  double* Pv = Cp + (size_t)f.NR * ld;            // A_{b,p} rows, sparse [ld][nz]
  double* Av = Pv + (size_t)ld * nz;              // A_bb rows, same pattern
  double* pk = Av + (size_t)ld * nz;              // pivot row and column [parity][2][ld]
  double* Es = pk + 4 * ld;
  double* K0s = Es + 2 * layer_width(g);
  int* Pc = reinterpret_cast<int*>(K0s + nd * nd);   // column of each sparse entry
  uint8_t* fl = reinterpret_cast<uint8_t*>(Pc + ld * nz);
  const int t = threadIdx.x;
  const bool act = t < R * C;   // the rest duplicate thread 0 and write nothing
  const int ti = act ? t / C : 0, tj = act ? t - (t / C) * C : 0;
  const int j = blockIdx.x, sys = blockIdx.y;
  const double* em = si.emod + (size_t)sys * g.nel;
  int jx, jy, jz;
  sub_coords(g, j, jx, jy, jz);
  for (int i = t; i < nd * nd; i += kThreads) K0s[i] = si.K0[i];
  for (int i = t; i < f.NR * ld; i += kThreads) Cp[i] = 0.0;
  for (int i = t; i < 4 * ld; i += kThreads) pk[i] = 0.0;
  const int mid = nblk / 2;
  const int nbot = si.twist ? nblk - 1 - mid : 0;
  double* TS = si.twist ? si.twist + ((size_t)sys * g.nsub + j) * ((size_t)nb * (nb + 1) / 2)
                        : nullptr;
  T* O = out + (size_t)sys * ostride + (size_t)j * nblk * tsh.tstride;
  double s[SR][SC];

  // owned entries to and from the dense LDS buffer
  auto store_s = [&]() {
    if (act)
#pragma unroll
      for (int a = 0; a < SR; ++a)
#pragma unroll
        for (int q = 0; q < SC; ++q) Cp[(ti + R * a) * ld + tj + C * q] = s[a][q];
  };

  // s = A_{cur,cur} - A_{cur,p} C_p A_{p,cur} (C_p in Cp) when withA, else
  // the product alone; element layers cur - 1 and cur are staged
  auto build = [&](int cur, int p, bool withA) {
    // an opaque copy of the thread index keeps the compiler from hoisting
    // the per-thread parts of the staging and sparse rows out of the block
    // loop, where they would hold registers through the elimination
    int tq = t;
    asm volatile("" : "+v"(tq));
    stage_layers<true>(si, jx, jy, jz, cur - 1, Es, fl, tq, em);
    __syncthreads();
    // sparse rows: row i couples to the nodes next to its node in a layer
    // (padding rows and outside nodes: column 0, value 0)
    for (int e = tq; e < ld * nz; e += kThreads) {
      const int i = e / nz, slot = e - (e / nz) * nz;
      const int node = i / d, c2 = slot % d, ns = slot / d;
      const int x = node % bn + ns % 3 - 1;
      const int y = (d == 3 ? node / bn : 0) + (d == 3 ? ns / 3 - 1 : 0);
      const bool in = i < nb && x >= 0 && x < bn && y >= 0 && y < (d == 3 ? bn : 1);
      const int k = in ? d * (x + bn * y) + c2 : 0;
      double v = 0.0, w = 0.0;
      if (in && !fl[nb + i]) {
        if (p >= 0 && !fl[(p - cur + 1) * nb + k])
          v = stencil_entry(g, cur * nb + i, p * nb + k, cur - 1, Es, K0s);
        if (withA)   // supported DOFs: decoupled, unit diagonal
          w = fl[nb + k] ? 0.0 : stencil_entry(g, cur * nb + i, cur * nb + k, cur - 1, Es, K0s);
      } else if (in && withA && k == i) {
        w = 1.0;
      }
      Pc[e] = k;
      Pv[e] = v;
      Av[e] = w;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < SR; ++a)
#pragma unroll
      for (int q = 0; q < SC; ++q) s[a][q] = 0.0;
    if (p >= 0) {
      // T[k][c] = sum_l C_p[k][l] A_{cur,p}[c][l]
#pragma unroll 1
      for (int z = 0; z < nz; ++z) {
        int l[SC];
        double pv[SC];
#pragma unroll
        for (int q = 0; q < SC; ++q) {
          l[q] = Pc[(tj + C * q) * nz + z];
          pv[q] = Pv[(tj + C * q) * nz + z];
        }
#pragma unroll
        for (int a = 0; a < SR; ++a)
#pragma unroll
          for (int q = 0; q < SC; ++q) s[a][q] += Cp[(ti + R * a) * ld + l[q]] * pv[q];
      }
      lds_barrier();
      store_s();
      lds_barrier();
      // A_{cur,p} T
#pragma unroll
      for (int a = 0; a < SR; ++a)
#pragma unroll
        for (int q = 0; q < SC; ++q) s[a][q] = 0.0;
#pragma unroll 1
      for (int z = 0; z < nz; ++z)
#pragma unroll
        for (int a = 0; a < SR; ++a) {
          const int r = ti + R * a;
          const double* Tk = Cp + Pc[r * nz + z] * ld + tj;
          const double pv = Pv[r * nz + z];
#pragma unroll
          for (int q = 0; q < SC; ++q) s[a][q] += pv * Tk[C * q];
        }
    }
    if (withA) {
      // A_{cur,cur} scattered into the cleared buffer (last read above)
      lds_barrier();
      for (int e = t; e < f.NR * ld; e += kThreads) Cp[e] = 0.0;
      lds_barrier();
      for (int e = t; e < nb * nz; e += kThreads) {
        const double w = Av[e];   // the nonzeros sit at distinct (row, column) places
        if (w != 0.0) Cp[(e / nz) * ld + Pc[e]] = w;
      }
      lds_barrier();
#pragma unroll
      for (int a = 0; a < SR; ++a)
#pragma unroll
        for (int q = 0; q < SC; ++q) s[a][q] = Cp[(ti + R * a) * ld + tj + C * q] - s[a][q];
    }
  };

  // s <- s^-1 in place by Gauss-Jordan elimination
  auto invert = [&]() {
#pragma unroll 1
    for (int k = 0; k < nb; ++k) {
      double* rowk = pk + (k & 1) * 2 * ld;
      double* colk = rowk + ld;
      const int ka = k / R, kr = k - ka * R, kq = k / C, kc = k - kq * C;
      if (act && ti == kr) {
#pragma unroll
        for (int a = 0; a < SR; ++a)
          if (a == ka)
#pragma unroll
            for (int q = 0; q < SC; ++q) rowk[tj + C * q] = s[a][q];
      }
      if (act && tj == kc) {
#pragma unroll
        for (int q = 0; q < SC; ++q)
          if (q == kq) {
#pragma unroll
            for (int a = 0; a < SR; ++a) {
              colk[ti + R * a] = s[a][q];
              s[a][q] = ti + R * a == k ? 1.0 : 0.0;
            }
          }
        if (ti == kr) rowk[k] = 1.0;
      }
      lds_barrier();
      double pv = colk[k];
      if (!(pv > 0.0)) {
        if (t == 0) flag[0] = 1;
        pv = 1.0;
      }
      const double inv = 1.0 / pv;
      double cr[SR], rc[SC];
#pragma unroll
      for (int a = 0; a < SR; ++a) {
        const int r = ti + R * a;
        cr[a] = r == k ? 1.0 - inv : colk[r] * inv;
      }
#pragma unroll
      for (int q = 0; q < SC; ++q) rc[q] = rowk[tj + C * q];
#pragma unroll
      for (int a = 0; a < SR; ++a)
#pragma unroll
        for (int q = 0; q < SC; ++q) s[a][q] = fma(-cr[a], rc[q], s[a][q]);
    }
  };

  for (int step = 0; step < nblk; ++step) {
    const bool bot = step < nbot;
    const int b = bot ? nblk - 1 - step : step - nbot;
    const bool first = step == 0 || step == nbot;
    __syncthreads();
    build(b, first ? -1 : (bot ? b + 1 : b - 1), true);
    if (!bot && nbot > 0 && b == mid) {
      // the lower half's term for the middle block
#pragma unroll
      for (int a = 0; a < SR; ++a)
#pragma unroll
        for (int q = 0; q < SC; ++q) {
          const int r = ti + R * a, c = tj + C * q;
          if (r < nb && c < nb)
            s[a][q] -= r >= c ? TS[(size_t)r * (r + 1) / 2 + c] : TS[(size_t)c * (c + 1) / 2 + r];
        }
    }
    invert();
    // C_b to LDS (the next block of the half reads it), then record b from
    // there in record order: the lower 4 x 4 tiles, diagonal tiles in full
    lds_barrier();
    store_s();
    lds_barrier();
    T* Rb = O + (size_t)b * tsh.tstride;
    constexpr int per = 16 / (int)sizeof(T);
    for (int o = t; o < tsh.tstride; o += kThreads) {
      const int gq = o / (tsh.nl * per), rem = o - gq * (tsh.nl * per);
      const int tau = rem / per, e = gq * per + (rem - (rem / per) * per);
      int I, J;
      tile_rc(tau, I, J);
      const int r = 4 * I + (e >> 2), c = 4 * J + (e & 3);
      Rb[o] = (T)(r < nb && c < nb ? Cp[r * ld + c] : 0.0);
    }
    if (bot && step + 1 == nbot) {
      // A_{mid,b} C_b A_{b,mid} (b = mid + 1) for the middle block
      __syncthreads();
      build(mid, b, false);
      if (act)
#pragma unroll
        for (int a = 0; a < SR; ++a)
#pragma unroll
          for (int q = 0; q < SC; ++q) {
            const int r = ti + R * a, c = tj + C * q;
            if (r < nb && c <= r) TS[(size_t)r * (r + 1) / 2 + c] = s[a][q];
          }
    }
  }
}

template <typename K>
void set_lds(K kernel) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();   // an unsupported size must not leave a stale error behind
}

}  // namespace

template <typename T>
void launch_factor(const double* A, T* out, int nmat, const BtriShape& sh, int* flag,
                   hipStream_t st, bool tiles, const StencilIn* si) {
  static bool attr = false;
  if (!attr) { set_lds(&k_btri_factor<T>); attr = true; }
  StencilIn s{};
  if (si) s = *si;
  const size_t lds = sizeof(double) * (2 * (size_t)sh.nb * lds_ld(sh.nb) + 4 * 256 +
                                       (si ? stencil_lds_elems(si->g) : 0));
  hipLaunchKernelGGL(k_btri_factor<T>, dim3(nmat), dim3(kThreads), lds, st, A, out, sh, flag,
                     tiles ? 1 : 0, s);
}

template <typename T, int NB>
void local_factor_as(const StencilIn& si, T* out, int* flag, int nsys, size_t ostride,
                     hipStream_t st) {
  static bool attr = false;
  if (!attr) { set_lds(&k_local_factor<T, NB>); attr = true; }
  hipLaunchKernelGGL((k_local_factor<T, NB>), dim3(si.g.nsub, nsys), dim3(kThreads),
                     local_factor_lds_bytes(si.g, lf_pick_shape(NB)), st, si, out, flag, ostride);
}

// block sizes with a compiled local factorisation: d (s + 1)^(d - 1) DOFs per
// node layer of a subdomain of s cells a side, 2-d s = 4 ... 40, 3-d s = 1 and 3 (odd 3-d
// blocks, s = 2 and 4, are refused by the preconditioner build)
#define TPCG_LF_SIZES(X) X(10) X(18) X(34) X(50) X(66) X(82) X(12) X(48)

bool local_factor_fits(const Geometry& g) {
  bool known = false;
#define TPCG_LF_KNOWN(n) known = known || g.nb == n;
  TPCG_LF_SIZES(TPCG_LF_KNOWN)
#undef TPCG_LF_KNOWN
  return known && local_factor_lds_bytes(g, lf_pick_shape(g.nb)) <= 160 * 1024;
}

template <typename T>
void launch_local_factor(const StencilIn& si, T* out, int* flag, int nsys, size_t ostride,
                         hipStream_t st) {
  switch (si.g.nb) {
#define TPCG_LF_CASE(n) \
  case n: local_factor_as<T, n>(si, out, flag, nsys, ostride, st); break;
    TPCG_LF_SIZES(TPCG_LF_CASE)
#undef TPCG_LF_CASE
    default: break;   // callers check local_factor_fits first
  }
}

template void launch_local_factor<double>(const StencilIn&, double*, int*, int, size_t,
                                          hipStream_t);
template void launch_local_factor<float>(const StencilIn&, float*, int*, int, size_t, hipStream_t);

template void launch_factor<double>(const double*, double*, int, const BtriShape&, int*,
                                    hipStream_t, bool, const StencilIn*);
template void launch_factor<float>(const double*, float*, int, const BtriShape&, int*,
                                   hipStream_t, bool, const StencilIn*);

#define TPCG_MULTI_CASE(V)                                                                  \
  case V: {                                                                                 \
    static bool attr = false;                                                               \
    if (!attr) { set_lds(&k_btri_solve_multi<V>); attr = true; }                            \
    hipLaunchKernelGGL(k_btri_solve_multi<V>, dim3(nmat), dim3(kThreads), lds, st, fac, sh, \
                       m, X, Y);                                                            \
    break;                                                                                  \
  }

void launch_solve_multi(const double* fac, const BtriShape& sh, int nmat, int m, const double* X,
                        double* Y, hipStream_t st) {
  const size_t lds = sizeof(double) * btri_solve16_lds_elems(sh);
  switch (stage_bucket(stage_regs_for<double>(sh.nb, sh.pe))) {
    TPCG_MULTI_CASE(2)
    TPCG_MULTI_CASE(5)
    TPCG_MULTI_CASE(10)
    TPCG_MULTI_CASE(16)
    TPCG_MULTI_CASE(24)
    TPCG_MULTI_CASE(36)
    default: break;
  }
}

#define TPCG_INV_CASE(V)                                                                     \
  case V: {                                                                                  \
    static bool attr = false;                                                                \
    if (!attr) { set_lds(&k_btri_inverse<V>); attr = true; }                                 \
    hipLaunchKernelGGL(k_btri_inverse<V>, dim3(nmat * chunks), dim3(kThreads), lds, st, fac, \
                       sh, chunks, Xinv);                                                    \
    break;                                                                                   \
  }

void launch_inverse(const double* fac, const BtriShape& sh, int nmat, double* Xinv,
                    hipStream_t st) {
  const int n = sh.nb * sh.nblk;
  const int chunks = (n + kMaxSub - 1) / kMaxSub;
  const size_t lds = sizeof(double) * btri_solve16_lds_elems(sh);
  switch (stage_bucket(stage_regs_for<double>(sh.nb, sh.pe))) {
    TPCG_INV_CASE(2)
    TPCG_INV_CASE(5)
    TPCG_INV_CASE(10)
    TPCG_INV_CASE(16)
    TPCG_INV_CASE(24)
    TPCG_INV_CASE(36)
    default: break;
  }
}

}  // namespace tpcg
