// Block-tridiagonal Cholesky factors and their triangular solves, one
// workgroup per matrix.
//
// A symmetric positive definite block-tridiagonal matrix with nblk diagonal
// blocks of size nb factors as A = L L^T with L block lower bidiagonal. The
// factor is stored per block row b as two dense nb x nb row-major matrices:
//   slot 0: D_b = L_bb^-1      (lower triangular; zeros above the diagonal)
//   slot 1: B_b = L_{b,b-1}    (B_0 unused)
// so that L y = r reads y_b = D_b (r_b - B_b y_{b-1}) and L^T x = y reads
// x_b = D_b^T (y_b - B_{b+1}^T x_{b+1}): every step is a dense product.
//
// Subdomain stiffness matrices in box order (node x fastest, then y, then z)
// are block tridiagonal with one node row (2D) or node layer (3D) per block.
#pragma once

#include "tpcg_internal.h"

namespace tpcg {

// odd leading dimension: conflict-free LDS columns and rows
__host__ __device__ inline int lds_ld(int nb) { return nb | 1; }

// Partial products of y = M v (trans = false) or y = M^T v (trans = true) for
// M in LDS (nb x nb, leading dimension ld). Thread t handles row (or column)
// t % nb over the chunk t / nb of the summation index and writes its partial
// to red[chunk * nb + row]. The caller sums the chunks after a barrier.
template <typename T>
__device__ inline void lds_gemv_parts(const T* M, int ld, int nb, const T* v, T* red, bool trans) {
  const int t = threadIdx.x;
  const int Q = kThreads / nb;
  const int L = (nb + Q - 1) / Q;
  const int i = t % nb, q = t / nb;
  if (q < Q) {
    const int c0 = q * L;
    const int c1 = min(nb, c0 + L);
    T acc = 0;
    if (!trans) {
      for (int c = c0; c < c1; ++c) acc += M[i * ld + c] * v[c];
    } else {
      for (int c = c0; c < c1; ++c) acc += M[c * ld + i] * v[c];
    }
    red[q * nb + i] = acc;
  }
}

template <typename T>
__device__ inline T lds_gemv_sum(const T* red, int nb, int i) {
  const int Q = kThreads / nb;
  T s = 0;
  for (int q = 0; q < Q; ++q) s += red[q * nb + i];
  return s;
}

// Register staging of one nb x nb matrix (nb even) read with 16-byte loads.
template <typename T, int MAXV>
struct MatStage {
  uint4 v[MAXV];

  __device__ inline void load(const T* src, int nv) {
    const uint4* s = reinterpret_cast<const uint4*>(src);
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const int idx = threadIdx.x + k * kThreads;
      if (idx < nv) v[k] = s[idx];
    }
  }

  __device__ inline void store(T* M, int ld, int nb, int nv) {
    constexpr int PER = 16 / sizeof(T);
    // element flat index f = PER * (t + 256 k): advance row/col incrementally
    const int step = PER * kThreads;
    const int dq = step / nb, dr = step - dq * nb;
    int f0 = PER * threadIdx.x;
    int row = f0 / nb, col = f0 - row * nb;
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const int idx = threadIdx.x + k * kThreads;
      if (idx < nv) {
        const T* e = reinterpret_cast<const T*>(&v[k]);
        int rr = row, cc = col;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          M[rr * ld + cc] = e[u];
          if (++cc == nb) { cc = 0; ++rr; }
        }
      }
      col += dr;
      row += dq;
      if (col >= nb) { col -= nb; ++row; }
    }
  }
};

template <typename T>
constexpr int stage_regs() { return sizeof(T) == 8 ? 18 : 9; }   // nb <= 96

// LDS bytes of btri_solve for block size nb
template <typename T>
inline size_t btri_solve_lds(int nb) {
  return sizeof(T) * ((size_t)nb * lds_ld(nb) + 2 * (size_t)nb + kThreads);
}

// Solve (L L^T) x = r for one block-tridiagonal factor `fac`
// ([nblk][2][nb][nb], T). rhs(b, i) returns element i of block b of r;
// out(b, i) is a T array slot that receives y (forward) and then x. The
// same thread reads back what it wrote, so no fence is needed.
template <typename T, typename Rhs, typename Out>
__device__ void btri_solve(const T* __restrict__ fac, int nb, int nblk, Rhs rhs, Out out,
                           unsigned char* smem) {
  const int ld = lds_ld(nb);
  T* M = reinterpret_cast<T*>(smem);
  T* va = M + (size_t)nb * ld;
  T* vb = va + nb;
  T* red = vb + nb;
  const int nv = nb * nb * (int)sizeof(T) / 16;
  const size_t msz = (size_t)nb * nb;
  const int t = threadIdx.x;
  // step s -> matrix: forward D0, B1, D1, ..., B_{n-1}, D_{n-1};
  // backward B_{n-1}, D_{n-2}, B_{n-2}, ..., B_1, D_0
  const int nf = 2 * nblk - 1;
  const int S = nf + 2 * (nblk - 1);
  auto mat = [&](int s) -> const T* {
    int b, slot;
    if (s < nf) { b = (s + 1) / 2; slot = (s & 1) ? 1 : 0; }
    else {
      const int u = s - nf;
      if ((u & 1) == 0) { b = nblk - 1 - u / 2; slot = 1; }
      else { b = nblk - 2 - u / 2; slot = 0; }
    }
    return fac + ((size_t)b * 2 + slot) * msz;
  };
  // vector needed in va at step s: forward D0 / B_b take r_b; backward
  // B_{b+1} takes y_b (b = nblk - 2 - u/2); the rest take none (-1)
  auto vec_kind = [&](int s, int& b) -> int {
    if (s < nf) {
      if (s == 0) { b = 0; return 0; }
      if (s & 1) { b = (s + 1) / 2; return 0; }
      return -1;
    }
    const int u = s - nf;
    if ((u & 1) == 0) { b = nblk - 2 - u / 2; return 1; }
    return -1;
  };
  MatStage<T, stage_regs<T>()> stage;
  T vreg = 0;
  {
    stage.load(mat(0), nv);
    int b;
    if (t < nb && vec_kind(0, b) == 0) vreg = (T)rhs(b, t);
  }
  for (int s = 0; s < S; ++s) {
    __syncthreads();
    stage.store(M, ld, nb, nv);
    int b = 0;
    const int kind = vec_kind(s, b);
    if (t < nb && kind >= 0) va[t] = vreg;
    if (s + 1 < S) {
      stage.load(mat(s + 1), nv);
      int b1 = 0;
      const int k1 = vec_kind(s + 1, b1);
      if (t < nb) {
        if (k1 == 0) vreg = (T)rhs(b1, t);
        else if (k1 == 1) vreg = out(b1, t);
      }
    }
    __syncthreads();
    if (s < nf) {
      const int bb = (s + 1) / 2;
      if (s & 1) {
        // t_b = r_b - B_b y_{b-1}
        lds_gemv_parts(M, ld, nb, vb, red, false);
        __syncthreads();
        if (t < nb) va[t] = va[t] - lds_gemv_sum(red, nb, t);
      } else {
        // y_b = D_b t_b
        lds_gemv_parts(M, ld, nb, va, red, false);
        __syncthreads();
        if (t < nb) {
          const T y = lds_gemv_sum(red, nb, t);
          vb[t] = y;
          out(bb, t) = y;
        }
        if (bb == nblk - 1) {
          // x_{n-1} = D_{n-1}^T y_{n-1}
          __syncthreads();
          lds_gemv_parts(M, ld, nb, vb, red, true);
          __syncthreads();
          if (t < nb) {
            const T x = lds_gemv_sum(red, nb, t);
            vb[t] = x;
            out(bb, t) = x;
          }
        }
      }
    } else {
      const int u = s - nf;
      if ((u & 1) == 0) {
        // s_b = y_b - B_{b+1}^T x_{b+1}
        lds_gemv_parts(M, ld, nb, vb, red, true);
        __syncthreads();
        if (t < nb) va[t] = va[t] - lds_gemv_sum(red, nb, t);
      } else {
        // x_b = D_b^T s_b
        const int bb = nblk - 2 - u / 2;
        lds_gemv_parts(M, ld, nb, va, red, true);
        __syncthreads();
        if (t < nb) {
          const T x = lds_gemv_sum(red, nb, t);
          vb[t] = x;
          out(bb, t) = x;
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace tpcg
