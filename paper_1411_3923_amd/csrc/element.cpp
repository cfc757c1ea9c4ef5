// Unit-modulus element stiffness K0 (Sec. 2.1: C = E(x) C0 with unit
// reference modulus; Sec. 2.2: K0 is the element matrix for E = 1).
//
// Bilinear unit-square element in plane stress (thickness 1) and trilinear
// unit-cube element, integrated with 2 Gauss points per axis, which is exact
// for these integrands (at most quadratic per axis).
#include <cmath>
#include <cstring>

namespace tpcg {

namespace {

// Derivatives of the d-linear shape functions on the unit cell at point x
// (coordinates in [0,1]^d). Corner a has coordinates bits (cx, cy, cz).
void shape_grad(int dim, const double* x, const int (*corner)[3], int nn, double (*dN)[3]) {
  for (int a = 0; a < nn; ++a) {
    for (int i = 0; i < dim; ++i) {
      double v = 1.0;
      for (int m = 0; m < dim; ++m) {
        const int c = corner[a][m];
        if (m == i) v *= (c ? 1.0 : -1.0);
        else v *= (c ? x[m] : 1.0 - x[m]);
      }
      dN[a][i] = v;
    }
  }
}

}  // namespace

void element_stiffness(int dim, double nu, double* K0) {
  static const int c2[4][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}};
  static const int c3[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                               {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
  const int nn = dim == 2 ? 4 : 8;
  const int nd = dim * nn;
  const int (*corner)[3] = dim == 2 ? c2 : c3;
  // Lame constants for E = 1; plane stress uses the reduced first constant.
  const double G = 1.0 / (2.0 * (1.0 + nu));
  const double lam = dim == 2 ? nu / (1.0 - nu * nu) : nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  std::memset(K0, 0, sizeof(double) * nd * nd);
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  const int npt = dim == 2 ? 4 : 8;
  const double w = 1.0 / npt;   // weights 1/2 per axis on [0, 1]
  for (int pt = 0; pt < npt; ++pt) {
    double x[3] = {g[pt & 1], g[(pt >> 1) & 1], g[(pt >> 2) & 1]};
    double dN[8][3];
    shape_grad(dim, x, corner, nn, dN);
    // energy density of (u_a e_i, u_b e_j):
    //   lam (d_i N_a)(d_j N_b) + G (d_j N_a)(d_i N_b) + G delta_ij grad N_a . grad N_b
    for (int a = 0; a < nn; ++a)
      for (int b = 0; b < nn; ++b) {
        double dot = 0.0;
        for (int m = 0; m < dim; ++m) dot += dN[a][m] * dN[b][m];
        for (int i = 0; i < dim; ++i)
          for (int j = 0; j < dim; ++j) {
            double v = lam * dN[a][i] * dN[b][j] + G * dN[a][j] * dN[b][i];
            if (i == j) v += G * dot;
            K0[(dim * a + i) * nd + dim * b + j] += w * v;
          }
      }
  }
}

}  // namespace tpcg
