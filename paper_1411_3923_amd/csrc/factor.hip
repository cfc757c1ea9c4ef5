// Batched block-tridiagonal Cholesky factorisation into the packed record
// format of btri.h, and the multi-right-hand-side solve used by the
// subspace iteration of the local eigenproblems.
#include "btri.h"

namespace tpcg {

namespace {

// One workgroup per matrix. Input: assembled blocks A[b][0] = A_bb,
// A[b][1] = A_{b,b-1} (FP64, row-major nb x nb). Output: packed records in T.
// flag[0] = 1 on a non-positive pivot (replaced by 1 so that the
// factorisation completes and the caller can report it).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_btri_factor(const double* __restrict__ A,
                                                         T* __restrict__ out, BtriShape sh,
                                                         int* __restrict__ flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nb = sh.nb, nblk = sh.nblk, pe = sh.pe;
  const int ld = lds_ld(nb);
  double* buf0 = reinterpret_cast<double*>(smem);
  double* buf1 = buf0 + (size_t)nb * ld;
  const size_t msz = (size_t)nb * nb;
  const double* F = A + (size_t)blockIdx.x * nblk * 2 * msz;
  T* O = out + (size_t)blockIdx.x * nblk * sh.bstride;
  const int t = threadIdx.x;
  const int ti = t >> 4, tj = t & 15;     // 16 x 16 thread tile
  double* Xa = buf0;                       // receives A_bb, then L_bb, then A_{b+1,b} -> B_{b+1}
  double* Yb = buf1;                       // B_b of the previous step, then D_b
  for (int b = 0; b < nblk; ++b) {
    const double* Ab = F + (size_t)b * 2 * msz;
    for (int e = t; e < nb * nb; e += kThreads) Xa[(e / nb) * ld + e % nb] = Ab[e];
    __syncthreads();
    if (b > 0) {
      // A_bb -= B_b B_b^T on the lower triangle
      for (int i = ti; i < nb; i += 16)
        for (int jj = tj; jj <= i; jj += 16) {
          double s = 0.0;
          for (int c = 0; c < nb; ++c) s += Yb[i * ld + c] * Yb[jj * ld + c];
          Xa[i * ld + jj] -= s;
        }
      __syncthreads();
    }
    // right-looking Cholesky of Xa (lower)
    for (int c = 0; c < nb; ++c) {
      if (t == 0) {
        double piv = Xa[c * ld + c];
        if (!(piv > 0.0)) {
          flag[0] = 1;
          piv = 1.0;
        }
        Xa[c * ld + c] = sqrt(piv);
      }
      __syncthreads();
      const double inv = 1.0 / Xa[c * ld + c];
      for (int i = c + 1 + t; i < nb; i += kThreads) Xa[i * ld + c] *= inv;
      __syncthreads();
      for (int i = c + 1 + ti; i < nb; i += 16) {
        const double lic = Xa[i * ld + c];
        for (int jj = c + 1 + tj; jj <= i; jj += 16) Xa[i * ld + jj] -= lic * Xa[jj * ld + c];
      }
      __syncthreads();
    }
    // D_b = L_bb^-1 into Yb, one column per thread (forward substitution)
    if (t < nb) {
      const int jj = t;
      for (int i = 0; i < nb; ++i) {
        double v;
        if (i < jj) v = 0.0;
        else if (i == jj) v = 1.0 / Xa[i * ld + i];
        else {
          double s = 0.0;
          for (int c = jj; c < i; ++c) s += Xa[i * ld + c] * Yb[c * ld + jj];
          v = -s / Xa[i * ld + i];
        }
        Yb[i * ld + jj] = v;
      }
    }
    __syncthreads();
    const bool last = b + 1 == nblk;
    if (!last) {
      // B_{b+1} = A_{b+1,b} D_b^T in place, thread i owns row i (right to left)
      const double* An = F + ((size_t)(b + 1) * 2 + 1) * msz;
      for (int e = t; e < nb * nb; e += kThreads) Xa[(e / nb) * ld + e % nb] = An[e];
      __syncthreads();
      if (t < nb) {
        const int i = t;
        for (int jj = nb - 1; jj >= 0; --jj) {
          double s = 0.0;
          for (int c = 0; c <= jj; ++c) s += Xa[i * ld + c] * Yb[jj * ld + c];
          Xa[i * ld + jj] = s;
        }
      }
      __syncthreads();
    }
    // record b: lower(D_b) | strict upper(B_{b+1}) | band of B_{b+1}
    T* R = O + (size_t)b * sh.bstride;
    for (int e = t; e < nb * nb; e += kThreads) {
      const int r = e / nb, c = e - (e / nb) * nb;
      const double v = c <= r ? Yb[r * ld + c] : (last ? 0.0 : Xa[r * ld + c]);
      R[e] = (T)v;
    }
    for (int e = t; e < nb * pe; e += kThreads) {
      const int r = e / pe, tt = e - (e / pe) * pe;
      const double v = (last || r - tt < 0) ? 0.0 : Xa[r * ld + r - tt];
      R[nb * nb + e] = (T)v;
    }
    for (int e = nb * nb + nb * pe + t; e < sh.bstride; e += kThreads) R[e] = (T)0;
    __syncthreads();
    if (!last) {
      // B_{b+1} stays in Xa for the next update; Yb receives the next block
      double* tmp = Xa;
      Xa = Yb;
      Yb = tmp;
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
  btri_solve<double, kMaxSub, MAXV>(
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
  btri_solve<double, kMaxSub, MAXV>(
      F, sh, nr, [&](int b, int i, int r) { return (b * nb + i == c0 + r) ? 1.0 : 0.0; },
      [&](int b, int i, int r) -> double& { return Xm[(size_t)(b * nb + i) * n + c0 + r]; },
      smem);
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
                   hipStream_t st) {
  static bool attr = false;
  if (!attr) { set_lds(&k_btri_factor<T>); attr = true; }
  const size_t lds = 2 * sizeof(double) * (size_t)sh.nb * lds_ld(sh.nb);
  hipLaunchKernelGGL(k_btri_factor<T>, dim3(nmat), dim3(kThreads), lds, st, A, out, sh, flag);
}

template void launch_factor<double>(const double*, double*, int, const BtriShape&, int*, hipStream_t);
template void launch_factor<float>(const double*, float*, int, const BtriShape&, int*, hipStream_t);

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
  const size_t lds = sizeof(double) * btri_solve_lds_elems(sh, m);
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
  const size_t lds = sizeof(double) * btri_solve_lds_elems(sh, kMaxSub);
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
