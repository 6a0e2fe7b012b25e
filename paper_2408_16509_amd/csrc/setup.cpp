// Host-side setup: element operators, periodic connectivity, geometry.
//
// Hexahedra (order p): Gauss--Legendre solution points and tensor face flux points;
// nodal Lagrange basis (barycentric form); DG correction functions of Huynh (the
// paper's FR reference), i.e. derivatives of the right/left Radau polynomials
// (P_{p+1} +- P_p)/2 folded into the 1-D derivative operator:
//     div along a line = Dh f + cp F_plus + cm F_minus,
//     Dh = D - gR' l(+1)^T - gL' l(-1)^T,  cp = gR',  cm = -gL'.
// Tetrahedra (order 4): the 35 alpha-optimised points printed in Fig. mesh(c);
// flux points are the surface solution points (Fig. mesh(b)), so interpolation is
// a gather; the correction is the DG lifting M^{-1} E with exact simplex integrals.
// All setup linear algebra is done in long double.
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <stdexcept>
#include <thread>
#include <unordered_map>

namespace frmi {

using ld = long double;

// ------------------------------------------------------------------ 1-D tools
static void legendre_and_deriv(int n, ld x, ld& P, ld& dP) {
  // three-term recurrence for P_k and P_k'
  ld p0 = 1, p1 = x, d0 = 0, d1 = 1;
  if (n == 0) { P = 1; dP = 0; return; }
  for (int k = 1; k < n; ++k) {
    ld p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    ld d2 = d0 + (2 * k + 1) * p1;        // P'_{k+1} = P'_{k-1} + (2k+1) P_k
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  P = p1; dP = d1;
}

static void gauss_legendre(int n, ld* x, ld* w) {
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    ld z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      ld P, dP;
      legendre_and_deriv(n, z, P, dP);
      ld dz = P / dP;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    ld P, dP;
    legendre_and_deriv(n, z, P, dP);
    x[n - 1 - i] = z;                       // increasing order
    w[n - 1 - i] = 2 / ((1 - z * z) * dP * dP);
  }
}

void build_hex_ops(int p, HexOps& o) {
  o = HexOps();
  o.p = p; o.n1 = p + 1; o.nsp = o.n1 * o.n1 * o.n1; o.nfpf = o.n1 * o.n1; o.nfp = 6 * o.nfpf;
  const int n = o.n1;
  ld x[kMaxP + 1], w[kMaxP + 1], bw[kMaxP + 1];
  gauss_legendre(n, x, w);
  for (int j = 0; j < n; ++j) {                // barycentric weights
    bw[j] = 1;
    for (int m = 0; m < n; ++m) if (m != j) bw[j] /= (x[j] - x[m]);
  }
  for (int side = 0; side < 2; ++side) {      // l_j(-1), l_j(+1)
    ld y = side ? 1.0L : -1.0L, den = 0;
    for (int m = 0; m < n; ++m) den += bw[m] / (y - x[m]);
    for (int j = 0; j < n; ++j) (side ? o.lp : o.lm)[j] = (double)(bw[j] / (y - x[j]) / den);
  }
  ld D[kMaxP + 1][kMaxP + 1] = {};
  for (int a = 0; a < n; ++a) {
    ld s = 0;
    for (int b = 0; b < n; ++b) if (b != a) { D[a][b] = bw[b] / bw[a] / (x[a] - x[b]); s += D[a][b]; }
    D[a][a] = -s;
  }
  for (int a = 0; a < n; ++a) {
    ld P1, dP1, P0, dP0;
    legendre_and_deriv(p + 1, x[a], P1, dP1);
    legendre_and_deriv(p, x[a], P0, dP0);
    ld gR = 0.5L * (dP1 + dP0);
    ld gL = 0.5L * ((p % 2 == 0) ? -1.0L : 1.0L) * (dP1 - dP0);
    o.cp[a] = (double)gR;
    o.cm[a] = (double)(-gL);
    o.x[a] = (double)x[a];
    o.w[a] = (double)w[a];
    for (int b = 0; b < n; ++b) o.D[a][b] = (double)D[a][b];
  }
  // fold the correction into the derivative (long double)
  ld lp[kMaxP + 1], lm[kMaxP + 1];
  for (int side = 0; side < 2; ++side) {
    ld y = side ? 1.0L : -1.0L, den = 0;
    for (int m = 0; m < n; ++m) den += bw[m] / (y - x[m]);
    for (int j = 0; j < n; ++j) (side ? lp : lm)[j] = bw[j] / (y - x[j]) / den;
  }
  for (int a = 0; a < n; ++a) {
    ld P1, dP1, P0, dP0;
    legendre_and_deriv(p + 1, x[a], P1, dP1);
    legendre_and_deriv(p, x[a], P0, dP0);
    ld gR = 0.5L * (dP1 + dP0);
    ld gL = 0.5L * ((p % 2 == 0) ? -1.0L : 1.0L) * (dP1 - dP0);
    for (int b = 0; b < n; ++b) o.Dh[a][b] = (double)(D[a][b] - gR * lp[b] - gL * lm[b]);
  }
  // orthonormal Legendre Vandermonde and its inverse V^T W (Gauss rule exact)
  for (int a = 0; a < n; ++a)
    for (int m = 0; m < n; ++m) {
      ld P, dP;
      legendre_and_deriv(m, x[a], P, dP);
      ld v = std::sqrt((2 * m + 1) / 2.0L) * P;
      o.Vm[a][m] = (double)v;
      o.Vmi[m][a] = (double)(v * w[a]);
    }
}

// ------------------------------------------------------------------ tetrahedron
// Fig. mesh(c): fourth-order alpha-optimised solution points (printed order).
static const double kA = 0.654653670707977, kB = 0.551583572090994, kC = 0.103167144181987;
static const double kTetPts[35][3] = {
    {-1, -1, -1}, {-kA, -1, -1}, {0, -1, -1}, {kA, -1, -1}, {1, -1, -1},
    {-1, -kA, -1}, {-kB, -kB, -1}, {kC, -kB, -1}, {kA, -kA, -1}, {-1, 0, -1},
    {-kB, kC, -1}, {0, 0, -1}, {-1, kA, -1}, {-kA, kA, -1}, {-1, 1, -1},
    {-1, -1, -kA}, {-kB, -1, -kB}, {kC, -1, -kB}, {kA, -1, -kA}, {-1, -kB, -kB},
    {-0.5, -0.5, -0.5}, {kC, -kB, -kB}, {-1, kC, -kB}, {-kB, kC, -kB}, {-1, kA, -kA},
    {-1, -1, 0}, {-kB, -1, kC}, {0, -1, 0}, {-1, -kB, kC}, {-kB, -kB, kC},
    {-1, 0, 0}, {-1, -1, kA}, {-kA, -1, kA}, {-1, -kA, kA}, {-1, -1, 1}};
// reference corners and faces (corner triples), outward unit normals
static const double kTetCorner[4][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}};
static const int kTetFace[4][3] = {{0, 1, 3}, {0, 1, 2}, {0, 2, 3}, {1, 2, 3}};
static const double kPyrCorner[5][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1}, {0, 0, 1}};
static const int kPyrFace[5][4] = {{0, 1, 2, 3}, {0, 1, 4, -1}, {1, 2, 4, -1}, {2, 3, 4, -1}, {3, 0, 4, -1}};
static const int kHexFaceCorners[6][4] = {{0, 3, 4, 7}, {1, 2, 5, 6}, {0, 1, 4, 5}, {2, 3, 6, 7}, {0, 1, 2, 3}, {4, 5, 6, 7}};

static ld factorial(int n) { ld r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }

template <int N>
static bool invert(ld (&A)[N][N], int n) {      // Gauss--Jordan, partial pivoting, in place
  int piv[N];
  ld B[N][N];
  for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) B[i][j] = (i == j);
  for (int c = 0; c < n; ++c) {
    int r = c;
    for (int i = c + 1; i < n; ++i) if (std::fabs(A[i][c]) > std::fabs(A[r][c])) r = i;
    if (std::fabs(A[r][c]) < 1e-300L) return false;
    piv[c] = r;
    for (int j = 0; j < n; ++j) { std::swap(A[c][j], A[r][j]); std::swap(B[c][j], B[r][j]); }
    ld d = A[c][c];
    for (int j = 0; j < n; ++j) { A[c][j] /= d; B[c][j] /= d; }
    for (int i = 0; i < n; ++i) if (i != c) {
      ld f = A[i][c];
      if (f == 0) continue;
      for (int j = 0; j < n; ++j) { A[i][j] -= f * A[c][j]; B[i][j] -= f * B[c][j]; }
    }
  }
  (void)piv;
  for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) A[i][j] = B[i][j];
  return true;
}

// normalised Jacobi polynomial P_n^{(a,0)} (orthonormal with weight (1-x)^a on [-1,1])
static ld jacobi(ld x, int alpha, int n) {
  const ld a = alpha, b = 0;
  std::vector<ld> P(n + 1);
  ld g0 = std::pow(2.0L, a + b + 1) / (a + b + 1) * std::tgamma(a + 1) * std::tgamma(b + 1) / std::tgamma(a + b + 1);
  P[0] = 1 / std::sqrt(g0);
  if (n == 0) return P[0];
  ld g1 = (a + 1) * (b + 1) / (a + b + 3) * g0;
  P[1] = ((a + b + 2) * x / 2 + (a - b) / 2) / std::sqrt(g1);
  ld aold = 2 / (2 + a + b) * std::sqrt((a + 1) * (b + 1) / (a + b + 3));
  for (int i = 1; i < n; ++i) {
    ld h1 = 2 * i + a + b;
    ld anew = 2 / (h1 + 2) * std::sqrt((i + 1) * (i + 1 + a + b) * (i + 1 + a) * (i + 1 + b) / (h1 + 1) / (h1 + 3));
    ld bnew = -(a * a - b * b) / h1 / (h1 + 2);
    P[i + 1] = 1 / anew * (-aold * P[i - 1] + (x - bnew) * P[i]);
    aold = anew;
  }
  return P[n];
}

// orthonormal modal basis of P_4 on the reference tet in collapsed coordinates
static ld pkd(const double* X, int i, int j, int k) {
  ld r = X[0], s = X[1], t = X[2];
  ld a = (std::fabs(s + t) > 1e-14L) ? 2 * (1 + r) / (-s - t) - 1 : -1;
  ld b = (std::fabs(t - 1) > 1e-14L) ? 2 * (1 + s) / (1 - t) - 1 : -1;
  ld c = t;
  return 2 * std::sqrt(2.0L) * jacobi(a, 0, i) * jacobi(b, 2 * i + 1, j) * std::pow(1 - b, i) *
         jacobi(c, 2 * (i + j) + 2, k) * std::pow(1 - c, i + j);
}

void build_tet_ops(TetOps& o) {
  constexpr int N = TetOps::nsp;
  for (int z = 0; z < N; ++z) for (int d = 0; d < 3; ++d) o.pts[z][d] = kTetPts[z][d];
  // faces and flux points (face-local order: ascending solution point index)
  int f_idx = 0;
  for (int f = 0; f < 4; ++f) {
    const double* A = kTetCorner[kTetFace[f][0]];
    const double* B = kTetCorner[kTetFace[f][1]];
    const double* C = kTetCorner[kTetFace[f][2]];
    double e1[3], e2[3], nv[3];
    for (int d = 0; d < 3; ++d) { e1[d] = B[d] - A[d]; e2[d] = C[d] - A[d]; }
    nv[0] = e1[1] * e2[2] - e1[2] * e2[1];
    nv[1] = e1[2] * e2[0] - e1[0] * e2[2];
    nv[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double nn = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    // orient outward: away from the centroid (-1/2,-1/2,-1/2)
    double dotc = 0;
    for (int d = 0; d < 3; ++d) dotc += nv[d] * (A[d] + 0.5);
    double sg = dotc > 0 ? 1.0 : -1.0;
    for (int d = 0; d < 3; ++d) o.nref[f][d] = sg * nv[d] / nn;
    for (int z = 0; z < N; ++z) {
      double dist = 0;
      for (int d = 0; d < 3; ++d) dist += (o.pts[z][d] - A[d]) * o.nref[f][d];
      if (std::fabs(dist) < 1e-12) { o.fp_src[f_idx] = z; o.fp_face[f_idx] = f; ++f_idx; }
    }
  }
  // monomials u^a v^b w^c of total degree <= 4 in unit-simplex coordinates u = (xi+1)/2
  std::vector<std::array<int, 3>> ex;
  for (int dsum = 0; dsum <= 4; ++dsum)
    for (int c = 0; c <= dsum; ++c)
      for (int b = 0; b <= dsum - c; ++b) ex.push_back({dsum - b - c, b, c});
  auto mono = [&](const double* X, int m) {
    ld u = (X[0] + 1) / 2, v = (X[1] + 1) / 2, w = (X[2] + 1) / 2;
    return std::pow(u, ex[m][0]) * std::pow(v, ex[m][1]) * std::pow(w, ex[m][2]);
  };
  auto dmono = [&](const double* X, int m, int d) {   // d/dxi_d = 1/2 d/du_d
    ld uu[3] = {(X[0] + 1) / 2.0L, (X[1] + 1) / 2.0L, (X[2] + 1) / 2.0L};
    int e = ex[m][d];
    if (e == 0) return (ld)0;
    ld r = 0.5L * e;
    for (int q = 0; q < 3; ++q) r *= std::pow(uu[q], q == d ? e - 1 : ex[m][q]);
    return r;
  };
  static ld Vm[N][N];
  for (int z = 0; z < N; ++z) for (int m = 0; m < N; ++m) Vm[z][m] = mono(o.pts[z], m);
  invert(Vm, N);                                  // C[m][j]: l_j = sum_m C[m][j] mono_m
  static ld Cm[N][N];
  for (int m = 0; m < N; ++m) for (int j = 0; j < N; ++j) Cm[m][j] = Vm[m][j];
  for (int d = 0; d < 3; ++d)
    for (int z = 0; z < N; ++z)
      for (int j = 0; j < N; ++j) {
        ld s = 0;
        for (int m = 0; m < N; ++m) s += dmono(o.pts[z], m, d) * Cm[m][j];
        o.D[d][z][j] = (double)s;
      }
  // exact simplex integrals (reference tet = 8 x unit simplex)
  auto simplex = [&](int a, int b, int c) { return 8 * factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3); };
  static ld M[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      ld s = 0;
      for (int m = 0; m < N; ++m)
        for (int q = 0; q < N; ++q)
          s += Cm[m][i] * Cm[q][j] * simplex(ex[m][0] + ex[q][0], ex[m][1] + ex[q][1], ex[m][2] + ex[q][2]);
      M[i][j] = s;
    }
  for (int j = 0; j < N; ++j) {
    ld s = 0;
    for (int m = 0; m < N; ++m) s += Cm[m][j] * simplex(ex[m][0], ex[m][1], ex[m][2]);
    o.weights[j] = (double)s;
  }
  // face mass matrices: E[src(q)][sigma(r)] = int_face phi_q phi_r dS
  static ld E[N][TetOps::nfp];
  for (int i = 0; i < N; ++i) for (int s = 0; s < TetOps::nfp; ++s) E[i][s] = 0;
  std::vector<std::array<int, 2>> ex2;
  for (int dsum = 0; dsum <= 4; ++dsum) for (int a = 0; a <= dsum; ++a) ex2.push_back({a, dsum - a});
  for (int f = 0; f < 4; ++f) {
    const double* A = kTetCorner[kTetFace[f][0]];
    const double* B = kTetCorner[kTetFace[f][1]];
    const double* C = kTetCorner[kTetFace[f][2]];
    ld e1[3], e2[3];
    for (int d = 0; d < 3; ++d) { e1[d] = B[d] - A[d]; e2[d] = C[d] - A[d]; }
    ld cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2], cz = e1[0] * e2[1] - e1[1] * e2[0];
    ld dA = std::sqrt(cx * cx + cy * cy + cz * cz);
    int ids[15], nq = 0;
    for (int s = 0; s < TetOps::nfp; ++s) if (o.fp_face[s] == f) ids[nq++] = s;
    // (s, t) face coordinates of the points: solve A + s e1 + t e2 = x by least squares (exact)
    ld st[15][2];
    ld g11 = 0, g12 = 0, g22 = 0;
    for (int d = 0; d < 3; ++d) { g11 += e1[d] * e1[d]; g12 += e1[d] * e2[d]; g22 += e2[d] * e2[d]; }
    ld det = g11 * g22 - g12 * g12;
    for (int q = 0; q < 15; ++q) {
      const double* X = o.pts[o.fp_src[ids[q]]];
      ld r1 = 0, r2 = 0;
      for (int d = 0; d < 3; ++d) { r1 += (X[d] - A[d]) * e1[d]; r2 += (X[d] - A[d]) * e2[d]; }
      st[q][0] = (g22 * r1 - g12 * r2) / det;
      st[q][1] = (g11 * r2 - g12 * r1) / det;
    }
    static ld Vf[15][15];
    for (int q = 0; q < 15; ++q)
      for (int m = 0; m < 15; ++m) Vf[q][m] = std::pow(st[q][0], ex2[m][0]) * std::pow(st[q][1], ex2[m][1]);
    invert(Vf, 15);
    for (int q = 0; q < 15; ++q)
      for (int r = 0; r < 15; ++r) {
        ld s = 0;
        for (int m = 0; m < 15; ++m)
          for (int n2 = 0; n2 < 15; ++n2) {
            int a = ex2[m][0] + ex2[n2][0], b = ex2[m][1] + ex2[n2][1];
            s += Vf[m][q] * Vf[n2][r] * factorial(a) * factorial(b) / factorial(a + b + 2);
          }
        E[o.fp_src[ids[q]]][ids[r]] = dA * s;
      }
  }
  invert(M, N);
  for (int i = 0; i < N; ++i)
    for (int s = 0; s < TetOps::nfp; ++s) {
      ld acc = 0;
      for (int j = 0; j < N; ++j) acc += M[i][j] * E[j][s];
      o.lift[i][s] = (double)acc;
    }
  // fold the collocated normal trace into the derivative:
  //   Dh_i[z][nu] = D_i[z][nu] - sum_{sigma: src(sigma) = nu} lift[z][sigma] n~_{face(sigma), i}
  for (int d = 0; d < 3; ++d)
    for (int z = 0; z < N; ++z)
      for (int nu = 0; nu < N; ++nu) {
        ld acc = o.D[d][z][nu];
        for (int sg = 0; sg < TetOps::nfp; ++sg)
          if (o.fp_src[sg] == nu) acc -= (ld)o.lift[z][sg] * o.nref[o.fp_face[sg]][d];
        o.Dh[d][z][nu] = (double)acc;
      }
  // orthonormal modal basis (graded by total degree)
  int m = 0;
  static ld Vp[N][N];
  for (int dsum = 0; dsum <= 4; ++dsum)
    for (int i = 0; i <= dsum; ++i)
      for (int j = 0; j <= dsum - i; ++j) {
        int k = dsum - i - j;
        for (int z = 0; z < N; ++z) Vp[z][m] = pkd(o.pts[z], i, j, k);
        o.deg[m] = dsum;
        ++m;
      }
  for (int z = 0; z < N; ++z) for (int q = 0; q < N; ++q) o.V[z][q] = (double)Vp[z][q];
  invert(Vp, N);
  for (int z = 0; z < N; ++z) for (int q = 0; q < N; ++q) o.Vinv[z][q] = (double)Vp[z][q];
}

// ------------------------------------------------------------------ geometry
// Hexahedra: x(xi) = sum_S c_S prod_{d in S} xi_d over the 8 subsets S of {0,1,2}
// (trilinear map of the VTK corners); coefficients stored as geo[comp*8 + S].
static const int kHexCorner[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                     {-1, -1, 1}, {1, -1, 1}, {1, 1, 1}, {-1, 1, 1}};
static const int kSubset[8] = {0, 1, 2, 4, 3, 5, 6, 7};   // S index -> bitmask: {},{0},{1},{2},{01},{02},{12},{012}

static void hex_coeffs(const double X[8][3], double c[24]) {
  for (int comp = 0; comp < 3; ++comp)
    for (int s = 0; s < 8; ++s) {
      int mask = kSubset[s];
      ld acc = 0;
      for (int n = 0; n < 8; ++n) {
        ld f = 1;
        for (int d = 0; d < 3; ++d) if (mask >> d & 1) f *= kHexCorner[n][d];
        acc += f * X[n][comp];
      }
      c[comp * 8 + s] = (double)(acc / 8);
    }
}

static void hex_map(const double c[24], const double xi[3], double x[3], double g[3][3]) {
  // g[k] = d x / d xi_k (column k of G)
  const double a = xi[0], b = xi[1], d = xi[2];
  for (int comp = 0; comp < 3; ++comp) {
    const double* q = c + comp * 8;
    x[comp] = q[0] + q[1] * a + q[2] * b + q[3] * d + q[4] * a * b + q[5] * a * d + q[6] * b * d + q[7] * a * b * d;
    g[0][comp] = q[1] + q[4] * b + q[5] * d + q[7] * b * d;
    g[1][comp] = q[2] + q[4] * a + q[6] * d + q[7] * a * d;
    g[2][comp] = q[3] + q[5] * a + q[6] * b + q[7] * a * b;
  }
}

static void cross(const double* u, const double* v, double* w) {
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
}

// reference points of hex flux points: face f = 2d + s, local q = t0 + n1 t1 over the
// two tangential axes in increasing order
static void hex_fp_ref(const HexOps& o, int f, int q, double xi[3]) {
  int d = f / 2, s = f % 2;
  int ta = (d == 0) ? 1 : 0, tb = (d == 2) ? 1 : 2;
  xi[d] = s ? 1.0 : -1.0;
  xi[ta] = o.x[q % o.n1];
  xi[tb] = o.x[q / o.n1];
}

// ------------------------------------------------------------------ connectivity
struct Key {
  int64_t k[3];
  bool operator==(const Key& o) const { return k[0] == o.k[0] && k[1] == o.k[1] && k[2] == o.k[2]; }
};
struct KeyHash {
  size_t operator()(const Key& a) const {
    uint64_t h = 1469598103934665603ULL;
    for (int i = 0; i < 3; ++i) { h ^= (uint64_t)a.k[i] + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2); }
    return (size_t)h;
  }
};

// Spread the low 21 bits of v so that bit i lands at bit 3i.
static uint64_t spread3(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

// Locality of a native order: over the 64-element tiles, the number of distinct tiles
// that hold the face neighbours of a tile's elements (faces matched by their corner
// ids; periodic pairs, whose corners are distinct images, are left out).
static int64_t tile_spread(const Block& b, int nc, const int64_t* enodes) {
  const int nf = nc == 8 ? 6 : 4, nfc = nc == 8 ? 4 : 3;
  std::unordered_map<Key, std::array<int64_t, 2>, KeyHash> faces;
  faces.reserve((size_t)b.n * nf);
  std::vector<std::vector<int64_t>> nbr((size_t)b.n);
  for (int64_t i = 0; i < b.n; ++i) {
    const int64_t e = b.elems[i];
    for (int f = 0; f < nf; ++f) {
      int64_t c[4] = {-1, -1, -1, -1};
      for (int k = 0; k < nfc; ++k) c[k] = enodes[e * 8 + (nc == 8 ? kHexFaceCorners[f][k] : kTetFace[f][k])];
      std::sort(c, c + nfc);
      Key key;   // distinct faces of a conforming mesh share at most two corners
      key.k[0] = c[0]; key.k[1] = c[1]; key.k[2] = c[2];
      auto it = faces.find(key);
      if (it == faces.end()) faces.emplace(key, std::array<int64_t, 2>{i, -1});
      else if (it->second[1] < 0) {
        it->second[1] = i;
        nbr[i].push_back(it->second[0]);
        nbr[it->second[0]].push_back(i);
      }
    }
  }
  int64_t total = 0;
  std::vector<int64_t> seen;
  for (int64_t t0 = 0; t0 < b.n; t0 += 64) {
    seen.clear();
    for (int64_t i = t0; i < std::min(b.n, t0 + 64); ++i)
      for (int64_t j : nbr[i]) seen.push_back(j / 64);
    std::sort(seen.begin(), seen.end());
    total += (int64_t)(std::unique(seen.begin(), seen.end()) - seen.begin());
  }
  return total;
}

// Renumber a block along the Morton (Z-order) curve of its element centroids, each
// coordinate quantised to 21 bits over the centroids' bounding box; ties keep the
// input order.  Elements that share faces then mostly share 64-element tiles, so
// the neighbour gathers of the face kernels touch few cache lines.
static void morton_order(Block& b, int nc, const double* xyz, const int64_t* enodes) {
  const int64_t n = b.n;
  if (n < 2) return;
  std::vector<double> cen((size_t)n * 3, 0.0);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < n; ++i) {
    const int64_t e = b.elems[i];
    for (int c = 0; c < nc; ++c)
      for (int d = 0; d < 3; ++d) cen[i * 3 + d] += xyz[enodes[e * 8 + c] * 3 + d] / nc;
    for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], cen[i * 3 + d]); hi[d] = std::max(hi[d], cen[i * 3 + d]); }
  }
  std::vector<std::pair<uint64_t, int64_t>> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t code = 0;
    for (int d = 0; d < 3; ++d) {
      const double span = hi[d] - lo[d];
      const double f = span > 0 ? (cen[i * 3 + d] - lo[d]) / span : 0.0;
      const uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, std::floor(f * 2097152.0)));
      code |= spread3(q) << d;
    }
    key[i] = {code, i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int64_t> elems((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    elems[i] = b.elems[key[i].second];
    b.canon_pos[i] = (int32_t)key[i].second;
  }
  b.elems.swap(elems);
}

std::string build_setup(int order, int64_t n_vert, const double* xyz, const double* period,
                        int64_t n_elem, const int32_t* etype, const int64_t* enodes,
                        int e_align, int elem_order, Setup& out, int& code) {
  code = 0;
  out = Setup();
  if (order < 1 || order > kMaxP) { code = 3; return "hexahedra support orders 1..4"; }
  bool has[3] = {false, false, false};
  const double span0 = [&] {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < n_vert; ++v)
      for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], xyz[v * 3 + d]); hi[d] = std::max(hi[d], xyz[v * 3 + d]); }
    return std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
  }();
  for (int64_t e = 0; e < n_elem; ++e) {
    if (etype[e] != kHex && etype[e] != kTet && etype[e] != kPyr) { code = 1; return "unknown element type"; }
    has[etype[e]] = true;
    int nc = etype[e] == kHex ? 8 : (etype[e] == kPyr ? 5 : 4);
    for (int c = 0; c < nc; ++c)
      if (enodes[e * 8 + c] < 0 || enodes[e * 8 + c] >= n_vert) { code = 1; return "corner index out of range"; }
    if (etype[e] == kPyr) {
      // affine base: corner 2 = corner 1 + corner 3 - corner 0
      double sk = 0;
      for (int d = 0; d < 3; ++d) {
        const double r = xyz[enodes[e * 8 + 2] * 3 + d] - xyz[enodes[e * 8 + 1] * 3 + d] -
                          xyz[enodes[e * 8 + 3] * 3 + d] + xyz[enodes[e * 8 + 0] * 3 + d];
        sk += r * r;
      }
      if (std::sqrt(sk) > 1e-10 * span0) { code = 2; return "pyramid base is not a parallelogram (the map must be affine)"; }
    }
  }
  if ((has[kTet] || has[kPyr]) && order != 4) { code = 3; return "tetrahedra and pyramids are supported at order 4 only"; }
  if (has[kPyr] && (has[kHex] || has[kTet]))
    { code = 3; return "pyramids are supported in meshes of pyramids only (no coupling to hexahedra or tetrahedra)"; }
  build_hex_ops(order, out.hex);
  if (has[kTet] || has[kPyr]) build_tet_ops(out.tet);
  if (has[kPyr]) build_pyr_ops(out.tet, out.pyr);
  const HexOps& H = out.hex;
  const TetOps& T = out.tet;
  const PyrOps& Y = out.pyr;
  // blocks
  int bidx[3] = {-1, -1, -1};
  for (int t = 0; t < 3; ++t) if (has[t]) {
    Block b;
    b.etype = t;
    for (int64_t e = 0; e < n_elem; ++e) if (etype[e] == t) b.elems.push_back(e);
    b.n = (int64_t)b.elems.size();
    b.canon_pos.resize(b.n);
    for (int64_t i = 0; i < b.n; ++i) b.canon_pos[i] = (int32_t)i;
    if (elem_order == 0 || elem_order == 2) {
      const int nc = t == kHex ? 8 : (t == kPyr ? 5 : 4);
      Block keep;
      if (elem_order == 0) { keep.n = b.n; keep.elems = b.elems; keep.canon_pos = b.canon_pos; }
      morton_order(b, nc, xyz, enodes);
      // automatic: keep the input order when its tiles are at least as compact
      if (elem_order == 0 && tile_spread(keep, nc, enodes) <= tile_spread(b, nc, enodes)) {
        b.elems.swap(keep.elems);
        b.canon_pos.swap(keep.canon_pos);
      }
    }
    b.e_pad = (b.n + e_align - 1) / e_align * e_align;
    b.nsp = t == kHex ? H.nsp : (t == kPyr ? PyrOps::nsp : T.nsp);
    b.nfp = t == kHex ? H.nfp : (t == kPyr ? PyrOps::nfp : T.nfp);
    b.nfaces = t == kHex ? 6 : (t == kPyr ? 5 : 4);
    b.nfpf = t == kHex ? H.nfpf : (t == kPyr ? 25 : T.nfpf);   // pyramids: the base's count (the largest)
    b.ngeo = t == kHex ? 24 : 10;
    b.geo.assign((size_t)b.ngeo * b.e_pad, 0.0);
    b.nbr_elem.assign((size_t)b.nfaces * b.e_pad, 0);
    b.nbr_info.assign((size_t)b.nfaces * b.e_pad, -1);
    b.sol_xyz.assign((size_t)b.n * b.nsp * 3, 0.0);
    bidx[t] = (int)out.blocks.size();
    out.blocks.push_back(std::move(b));
  }
  // ---- geometry, Jacobian check, solution points
  for (auto& b : out.blocks) {
    for (int64_t le = 0; le < b.e_pad; ++le) {
      int64_t e = b.elems[le < b.n ? le : 0];
      if (b.etype == kHex) {
        double X[8][3], c[24];
        for (int n = 0; n < 8; ++n) for (int d = 0; d < 3; ++d) X[n][d] = xyz[enodes[e * 8 + n] * 3 + d];
        hex_coeffs(X, c);
        for (int g = 0; g < 24; ++g) b.geo[(size_t)g * b.e_pad + le] = c[g];
        if (le >= b.n) continue;
        for (int z = 0; z < H.nsp + H.nfp; ++z) {
          double xi[3], x[3], G[3][3], cr[3];
          if (z < H.nsp) { xi[0] = H.x[z % H.n1]; xi[1] = H.x[(z / H.n1) % H.n1]; xi[2] = H.x[z / (H.n1 * H.n1)]; }
          else hex_fp_ref(H, (z - H.nsp) / H.nfpf, (z - H.nsp) % H.nfpf, xi);
          hex_map(c, xi, x, G);
          cross(G[1], G[2], cr);
          double J = G[0][0] * cr[0] + G[0][1] * cr[1] + G[0][2] * cr[2];
          if (!(J > 0)) { code = 2; return "element with J <= 0"; }
          if (z < H.nsp)
            for (int d = 0; d < 3; ++d) b.sol_xyz[((size_t)b.canon_pos[le] * b.nsp + z) * 3 + d] = x[d];
        }
      } else if (b.etype == kPyr) {
        double X[5][3];
        for (int n = 0; n < 5; ++n) for (int d = 0; d < 3; ++d) X[n][d] = xyz[enodes[e * 8 + n] * 3 + d];
        double g[3][3];   // dx/dxi_k: (X1 - X0)/2, (X3 - X0)/2, (X4 - base centre)/2
        for (int d = 0; d < 3; ++d) {
          g[0][d] = 0.5 * (X[1][d] - X[0][d]);
          g[1][d] = 0.5 * (X[3][d] - X[0][d]);
          g[2][d] = 0.5 * (X[4][d] - 0.5 * (X[1][d] + X[3][d]));
        }
        double S[3][3];
        cross(g[1], g[2], S[0]);
        cross(g[2], g[0], S[1]);
        cross(g[0], g[1], S[2]);
        double J = g[0][0] * S[0][0] + g[0][1] * S[0][1] + g[0][2] * S[0][2];
        if (le < b.n && !(J > 0)) { code = 2; return "element with J <= 0"; }
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) b.geo[(size_t)(i * 3 + j) * b.e_pad + le] = S[i][j];
        b.geo[(size_t)9 * b.e_pad + le] = J;
        if (le >= b.n) continue;
        for (int z = 0; z < PyrOps::nsp; ++z)
          for (int d = 0; d < 3; ++d) {
            double x = X[0][d];
            for (int k = 0; k < 3; ++k) x += (Y.pts[z][k] + 1.0) * g[k][d];
            b.sol_xyz[((size_t)b.canon_pos[le] * b.nsp + z) * 3 + d] = x;
          }
      } else {
        double X[4][3];
        for (int n = 0; n < 4; ++n) for (int d = 0; d < 3; ++d) X[n][d] = xyz[enodes[e * 8 + n] * 3 + d];
        double g[3][3];   // columns: xi0 -> corner1, xi1 -> corner3, xi2 -> corner2
        for (int d = 0; d < 3; ++d) {
          g[0][d] = 0.5 * (X[1][d] - X[0][d]);
          g[1][d] = 0.5 * (X[3][d] - X[0][d]);
          g[2][d] = 0.5 * (X[2][d] - X[0][d]);
        }
        double S[3][3];
        cross(g[1], g[2], S[0]);
        cross(g[2], g[0], S[1]);
        cross(g[0], g[1], S[2]);
        double J = g[0][0] * S[0][0] + g[0][1] * S[0][1] + g[0][2] * S[0][2];
        if (le < b.n && !(J > 0)) { code = 2; return "element with J <= 0"; }
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) b.geo[(size_t)(i * 3 + j) * b.e_pad + le] = S[i][j];
        b.geo[(size_t)9 * b.e_pad + le] = J;
        if (le >= b.n) continue;
        for (int z = 0; z < T.nsp; ++z)
          for (int d = 0; d < 3; ++d) {
            double x = X[0][d];
            for (int k = 0; k < 3; ++k) x += (T.pts[z][k] + 1.0) * g[k][d];
            b.sol_xyz[((size_t)b.canon_pos[le] * b.nsp + z) * 3 + d] = x;
          }
      }
    }
  }
  // ---- face matching
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < n_vert; ++v)
    for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], xyz[v * 3 + d]); hi[d] = std::max(hi[d], xyz[v * 3 + d]); }
  double span = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
  const double scale = 1e-8 * span;
  auto face_nc = [&](const Block& b, int f) { return b.etype == kHex ? 4 : (b.etype == kPyr ? (f == 0 ? 4 : 3) : 3); };
  auto face_nq = [&](const Block& b, int f) { return b.etype == kPyr ? Y.face_off[f + 1] - Y.face_off[f] : b.nfpf; };
  auto face_centroid = [&](const Block& b, int64_t le, int f, double c[3]) {
    int64_t e = b.elems[le];
    int nc = face_nc(b, f);
    c[0] = c[1] = c[2] = 0;
    for (int k = 0; k < nc; ++k) {
      int corner = b.etype == kHex ? kHexFaceCorners[f][k] : (b.etype == kPyr ? kPyrFace[f][k] : kTetFace[f][k]);
      for (int d = 0; d < 3; ++d) c[d] += xyz[enodes[e * 8 + corner] * 3 + d];
    }
    for (int d = 0; d < 3; ++d) c[d] /= nc;
  };
  std::unordered_map<Key, std::vector<std::array<int64_t, 3>>, KeyHash> buckets;
  buckets.reserve((size_t)n_elem * 6);
  for (int bi = 0; bi < (int)out.blocks.size(); ++bi) {
    const Block& b = out.blocks[bi];
    for (int64_t le = 0; le < b.n; ++le)
      for (int f = 0; f < b.nfaces; ++f) {
        double c[3];
        face_centroid(b, le, f, c);
        Key k;
        for (int d = 0; d < 3; ++d) {
          if (period[d] > 0) {
            double r = std::fmod(c[d], period[d]);
            if (r < 0) r += period[d];
            int64_t n = std::llround(period[d] / scale);
            k.k[d] = std::llround(r / scale) % n;
          } else {
            k.k[d] = std::llround(c[d] / scale);
          }
        }
        buckets[k].push_back({bi, le, f});
      }
  }
  // flux point physical coordinates of one face
  auto face_points = [&](const Block& b, int64_t le, int f, std::vector<std::array<double, 3>>& P) {
    P.resize(face_nq(b, f));
    int64_t e = b.elems[le];
    for (int q = 0; q < (int)P.size(); ++q) {
      if (b.etype == kPyr) {
        const double* xi = Y.fpts[Y.face_off[f] + q];
        double X[5][3];
        for (int n = 0; n < 5; ++n) for (int d = 0; d < 3; ++d) X[n][d] = xyz[enodes[e * 8 + n] * 3 + d];
        for (int d = 0; d < 3; ++d)
          P[q][d] = X[0][d] + 0.5 * (xi[0] + 1) * (X[1][d] - X[0][d]) + 0.5 * (xi[1] + 1) * (X[3][d] - X[0][d]) +
                    0.5 * (xi[2] + 1) * (X[4][d] - 0.5 * (X[1][d] + X[3][d]));
      } else if (b.etype == kHex) {
        double c[24], xi[3], x[3], G[3][3];
        for (int g = 0; g < 24; ++g) c[g] = b.geo[(size_t)g * b.e_pad + le];
        hex_fp_ref(H, f, q, xi);
        hex_map(c, xi, x, G);
        P[q] = {x[0], x[1], x[2]};
      } else {
        int s = f * 15 + q;
        const double* xi = T.pts[T.fp_src[s]];
        double X[4][3];
        for (int n = 0; n < 4; ++n) for (int d = 0; d < 3; ++d) X[n][d] = xyz[enodes[e * 8 + n] * 3 + d];
        for (int d = 0; d < 3; ++d)
          P[q][d] = X[0][d] + 0.5 * (xi[0] + 1) * (X[1][d] - X[0][d]) + 0.5 * (xi[1] + 1) * (X[3][d] - X[0][d]) +
                    0.5 * (xi[2] + 1) * (X[2][d] - X[0][d]);
      }
    }
  };
  // outward scaled normal at the reference face centre
  auto face_normal = [&](const Block& b, int64_t le, int f, double nv[3]) {
    if (b.etype == kHex) {
      double c[24], xi[3] = {0, 0, 0}, x[3], G[3][3];
      for (int g = 0; g < 24; ++g) c[g] = b.geo[(size_t)g * b.e_pad + le];
      int d = f / 2;
      xi[d] = (f % 2) ? 1.0 : -1.0;
      hex_map(c, xi, x, G);
      cross(G[(d + 1) % 3], G[(d + 2) % 3], nv);
      double sg = (f % 2) ? 1.0 : -1.0;
      for (int k = 0; k < 3; ++k) nv[k] *= sg;
    } else {
      const double* nr = b.etype == kPyr ? Y.nref[f] : T.nref[f];
      for (int j = 0; j < 3; ++j) {
        nv[j] = 0;
        for (int i = 0; i < 3; ++i) nv[j] += b.geo[(size_t)(i * 3 + j) * b.e_pad + le] * nr[i];
      }
    }
  };
  std::map<std::vector<int32_t>, int> perm_ids;
  std::vector<std::vector<int32_t>> perms;
  auto perm_id = [&](const std::vector<int32_t>& p) {
    auto it = perm_ids.find(p);
    if (it != perm_ids.end()) return it->second;
    int id = (int)perms.size();
    perm_ids[p] = id;
    perms.push_back(p);
    return id;
  };
  std::vector<std::array<double, 3>> PA, PB;
  for (auto& kv : buckets) {
    auto& lst = kv.second;
    if (lst.size() != 2) { code = 2; return "face without exactly one partner (unpaired or non-conforming mesh)"; }
    Block& A = out.blocks[lst[0][0]];
    Block& B = out.blocks[lst[1][0]];
    int64_t ea = lst[0][1], eb = lst[1][1];
    int fa = (int)lst[0][2], fb = (int)lst[1][2];
    if (A.etype != B.etype) { code = 3; return "hexahedron-tetrahedron interfaces need pyramids (not supported)"; }
    if (face_nq(A, fa) != face_nq(B, fb)) { code = 2; return "matched faces of different kinds"; }
    face_points(A, ea, fa, PA);
    face_points(B, eb, fb, PB);
    double ca[3], cb[3], sh[3];
    face_centroid(A, ea, fa, ca);
    face_centroid(B, eb, fb, cb);
    for (int d = 0; d < 3; ++d) {
      double dd = ca[d] - cb[d];
      double w = dd;
      if (period[d] > 0) w = dd - period[d] * std::nearbyint(dd / period[d]);
      sh[d] = dd - w;
    }
    int nq = face_nq(A, fa);
    std::vector<int32_t> pa(nq), pb(nq, -1);
    for (int q = 0; q < nq; ++q) {
      int best = -1;
      double bd = 1e300;
      for (int r = 0; r < nq; ++r) {
        double d2 = 0;
        for (int d = 0; d < 3; ++d) { double t = PA[q][d] - PB[r][d] - sh[d]; d2 += t * t; }
        if (d2 < bd) { bd = d2; best = r; }
      }
      if (std::sqrt(bd) > 1e-8 * span || pb[best] != -1) { code = 2; return "flux points of matched faces do not conform"; }
      pa[q] = best;
      pb[best] = q;
    }
    double nv[3];
    face_normal(A, ea, fa, nv);
    double mx = std::max({std::fabs(nv[0]), std::fabs(nv[1]), std::fabs(nv[2])});
    int dom = 0;
    while (std::fabs(nv[dom]) < (1 - 1e-6) * mx) ++dom;
    int a_left = nv[dom] > 0 ? 1 : 0;
    int oa = perm_id(pa), ob = perm_id(pb);
    if (oa > 511 || ob > 511) { code = 3; return "too many distinct face orientations"; }
    A.nbr_elem[(size_t)fa * A.e_pad + ea] = (int32_t)eb;
    A.nbr_info[(size_t)fa * A.e_pad + ea] = fb | (oa << 3) | (a_left << 12);
    B.nbr_elem[(size_t)fb * B.e_pad + eb] = (int32_t)ea;
    B.nbr_info[(size_t)fb * B.e_pad + eb] = fa | (ob << 3) | ((1 - a_left) << 12);
  }
  // padding lanes copy element 0's connectivity (in-bounds, results discarded)
  for (auto& b : out.blocks) {
    for (int f = 0; f < b.nfaces; ++f)
      for (int64_t le = 0; le < b.e_pad; ++le) {
        size_t i = (size_t)f * b.e_pad + le;
        if (le >= b.n) { b.nbr_elem[i] = b.nbr_elem[(size_t)f * b.e_pad]; b.nbr_info[i] = b.nbr_info[(size_t)f * b.e_pad]; }
        if (b.nbr_info[i] < 0) { code = 2; return "unpaired face"; }
      }
  }
  out.n_orient = (int)perms.size();
  out.perm_stride = 0;
  for (auto& p : perms) out.perm_stride = std::max(out.perm_stride, (int)p.size());
  out.orient_perm.assign((size_t)std::max(out.n_orient, 1) * std::max(out.perm_stride, 1), 0);
  for (int i = 0; i < out.n_orient; ++i)
    for (size_t q = 0; q < perms[i].size(); ++q) out.orient_perm[(size_t)i * out.perm_stride + q] = perms[i][q];
  (void)bidx;
  return "";
}

}  // namespace frmi

namespace frmi {

// ------------------------------------------------------------------ curved hexahedra
// Sec. "Curved elements": per-point metric terms of curved elements, formed either as
// cross products of the exact map's derivatives or in the conservative (curl) form,
// whose discrete divergence vanishes so that a uniform stream stays uniform.
//
// Conservative form, with (n, m, l) cyclic: S_rn = J dxi_r/dx_n = -[curl_xi V^(n)]_r,
// V^(n) = I(x_l grad_xi x_m), I the tensor interpolant on the (p+1)^3 Gauss--Lobatto
// points.  Here V^(n) is sampled at the Lobatto grid, differentiated there with the
// 1-D Lobatto derivative matrix (exact for the interpolant), the curl formed at the
// grid, and the resulting Q_p polynomial evaluated at the Gauss solution points and
// the flux points (on a face xi_d = +-1 the Lobatto end nodes are face values, so
// only the tangential interpolation remains).

// Gauss--Lobatto nodes of n = 2..5 points, closed forms.
static void gll_points(int n, ld* y) {
  y[0] = -1;
  y[n - 1] = 1;
  if (n == 3) y[1] = 0;
  if (n == 4) { y[1] = -1 / sqrtl(5.0L); y[2] = -y[1]; }
  if (n == 5) { y[1] = -sqrtl(3.0L / 7.0L); y[2] = 0; y[3] = -y[1]; }
}

// Values and derivatives of the n Lagrange polynomials on `nodes` at x.
static void lagrange_1d(const ld* nodes, int n, ld x, ld* val, ld* der) {
  for (int j = 0; j < n; ++j) {
    ld v = 1, dsum = 0;
    for (int m = 0; m < n; ++m) {
      if (m == j) continue;
      v *= (x - nodes[m]) / (nodes[j] - nodes[m]);
    }
    for (int k = 0; k < n; ++k) {
      if (k == j) continue;
      ld t = 1 / (nodes[j] - nodes[k]);
      for (int m = 0; m < n; ++m)
        if (m != j && m != k) t *= (x - nodes[m]) / (nodes[j] - nodes[m]);
      dsum += t;
    }
    val[j] = v;
    der[j] = dsum;
  }
}

std::string build_curved_hex(int q, int metric, const double* xyz, const int64_t* ho, Setup& s, int& code) {
  code = 0;
  Block* bp = nullptr;
  for (auto& b : s.blocks) if (b.etype == kHex) bp = &b;
  if (!bp) { code = 1; return "no hexahedra"; }
  Block& b = *bp;
  const HexOps& H = s.hex;
  const int n1 = H.n1, nsp = H.nsp, nq = q + 1, NQ = nq * nq * nq, NG = n1 * n1 * n1;
  const int rows = 10 * nsp + 3 * H.nfp;
  b.cmet.assign((size_t)rows * b.e_pad, 0.0);
  // 1-D tables in long double, used in double
  ld gn[5], y[5], xg[5], t1[5], t2[5];
  for (int i = 0; i < nq; ++i) gn[i] = -1 + 2 * (ld)i / q;
  gll_points(n1, y);
  for (int i = 0; i < n1; ++i) xg[i] = H.x[i];
  double Dg[5][5], Ig[5][5];           // Lobatto derivative matrix; Lobatto basis at the Gauss points
  double Lly[5][5], dLy[5][5], Llx[5][5], dLx[5][5], Lle[2][5], dLe[2][5];   // geometry basis
  for (int a = 0; a < n1; ++a) {
    lagrange_1d(y, n1, y[a], t1, t2);
    for (int j = 0; j < n1; ++j) Dg[a][j] = (double)t2[j];
    lagrange_1d(y, n1, xg[a], t1, t2);
    for (int j = 0; j < n1; ++j) Ig[a][j] = (double)t1[j];
    lagrange_1d(gn, nq, y[a], t1, t2);
    for (int j = 0; j < nq; ++j) { Lly[a][j] = (double)t1[j]; dLy[a][j] = (double)t2[j]; }
    lagrange_1d(gn, nq, xg[a], t1, t2);
    for (int j = 0; j < nq; ++j) { Llx[a][j] = (double)t1[j]; dLx[a][j] = (double)t2[j]; }
  }
  for (int sd = 0; sd < 2; ++sd) {
    lagrange_1d(gn, nq, sd ? 1 : -1, t1, t2);
    for (int j = 0; j < nq; ++j) { Lle[sd][j] = (double)t1[j]; dLe[sd][j] = (double)t2[j]; }
  }
  auto det3 = [](const double G[3][3]) {
    return G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) - G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
           G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
  };
  // exact metric row r = g_{r+1} x g_{r+2}, g_j = column j of G
  auto cross_rows = [](const double G[3][3], double S[3][3]) {
    for (int r = 0; r < 3; ++r) {
      const int a = (r + 1) % 3, c = (r + 2) % 3;
      S[r][0] = G[1][a] * G[2][c] - G[2][a] * G[1][c];
      S[r][1] = G[2][a] * G[0][c] - G[0][a] * G[2][c];
      S[r][2] = G[0][a] * G[1][c] - G[1][a] * G[0][c];
    }
  };
  auto put = [&](int64_t le, int row, double v) { b.cmet[(size_t)row * b.e_pad + le] = v; };
  // elements [lo, hi): all buffers local, so threads share nothing but the outputs
  auto work = [&](int64_t lo, int64_t hi, std::string& err) {
    std::vector<double> X((size_t)NQ * 3), V((size_t)3 * NG * 3), Ja((size_t)NG * 9), T1((size_t)NG * 9),
        T2((size_t)NG * 9);
    // x and G (G[c][j] = d x_c / d xi_j) from 1-D tables of the three coordinates
    auto geo_at = [&](const double* L0, const double* D0, const double* L1, const double* D1, const double* L2,
                      const double* D2, double x[3], double G[3][3]) {
      for (int c = 0; c < 3; ++c) { x[c] = 0; G[c][0] = G[c][1] = G[c][2] = 0; }
      for (int k = 0; k < nq; ++k)
        for (int j = 0; j < nq; ++j) {
          const double ljk = L1[j] * L2[k], djk = D1[j] * L2[k], ljd = L1[j] * D2[k];
          for (int i = 0; i < nq; ++i) {
            const double* Xn = &X[(size_t)(i + nq * (j + nq * k)) * 3];
            const double w = L0[i] * ljk, w0 = D0[i] * ljk, w1 = L0[i] * djk, w2 = L0[i] * ljd;
            for (int c = 0; c < 3; ++c) {
              x[c] += w * Xn[c];
              G[c][0] += w0 * Xn[c];
              G[c][1] += w1 * Xn[c];
              G[c][2] += w2 * Xn[c];
            }
          }
        }
    };
    for (int64_t le = lo; le < hi; ++le) {
      const int64_t e = b.elems[le];
      for (int n = 0; n < NQ; ++n)
        for (int c = 0; c < 3; ++c) X[(size_t)n * 3 + c] = xyz[ho[e * NQ + n] * 3 + c];
      if (metric == 0) {
        // the factor x_l relative to node 0: no change in exact arithmetic for q <= p
        // (the interpolated grad x_m has zero curl), no cancellation of |x| against h^2
        double X0[3] = {X[0], X[1], X[2]};
        // V^(n)[node][k] = (x_l - x0_l) d x_m / d xi_k at the Lobatto grid
        for (int c = 0; c < n1; ++c)
          for (int bb = 0; bb < n1; ++bb)
            for (int a = 0; a < n1; ++a) {
              double x[3], G[3][3];
              geo_at(Lly[a], dLy[a], Lly[bb], dLy[bb], Lly[c], dLy[c], x, G);
              const int node = a + n1 * (bb + n1 * c);
              for (int n = 0; n < 3; ++n) {
                const int m = (n + 1) % 3, l = (n + 2) % 3;
                for (int k = 0; k < 3; ++k) V[((size_t)n * NG + node) * 3 + k] = (x[l] - X0[l]) * G[m][k];
              }
            }
        // curl at the grid: Ja[node][r*3 + n] = -(d_a V_b - d_b V_a), (r, a, b) cyclic
        for (int c = 0; c < n1; ++c)
          for (int bb = 0; bb < n1; ++bb)
            for (int a = 0; a < n1; ++a) {
              const int node = a + n1 * (bb + n1 * c);
              const int idx[3] = {a, bb, c};
              const int stride[3] = {1, n1, n1 * n1};
              for (int n = 0; n < 3; ++n) {
                double dV[3][3];   // dV[ax][k] = d V_k / d xi_ax at this node
                for (int ax = 0; ax < 3; ++ax) {
                  const int base = node - idx[ax] * stride[ax];
                  for (int k = 0; k < 3; ++k) {
                    double acc = 0;
                    for (int t = 0; t < n1; ++t) acc += Dg[idx[ax]][t] * V[((size_t)n * NG + base + t * stride[ax]) * 3 + k];
                    dV[ax][k] = acc;
                  }
                }
                for (int r = 0; r < 3; ++r) {
                  const int ra = (r + 1) % 3, rb = (r + 2) % 3;
                  Ja[(size_t)node * 9 + r * 3 + n] = -(dV[ra][rb] - dV[rb][ra]);
                }
              }
            }
        // the Q_p polynomial at the Gauss solution points, one axis at a time
        for (int c = 0; c < n1; ++c)
          for (int bb = 0; bb < n1; ++bb)
            for (int i = 0; i < n1; ++i)
              for (int r = 0; r < 9; ++r) {
                double acc = 0;
                for (int a = 0; a < n1; ++a) acc += Ig[i][a] * Ja[(size_t)(a + n1 * (bb + n1 * c)) * 9 + r];
                T1[(size_t)(i + n1 * (bb + n1 * c)) * 9 + r] = acc;
              }
        for (int c = 0; c < n1; ++c)
          for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i)
              for (int r = 0; r < 9; ++r) {
                double acc = 0;
                for (int bb = 0; bb < n1; ++bb) acc += Ig[j][bb] * T1[(size_t)(i + n1 * (bb + n1 * c)) * 9 + r];
                T2[(size_t)(i + n1 * (j + n1 * c)) * 9 + r] = acc;
              }
      }
      // solution points: S rows, 1/J, physical coordinates
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            const int pt = i + n1 * (j + n1 * k);
            double x[3], G[3][3], S[3][3];
            geo_at(Llx[i], dLx[i], Llx[j], dLx[j], Llx[k], dLx[k], x, G);
            const double J = det3(G);
            if (!(J > 0)) { err = "curved element with J <= 0"; return; }
            if (metric == 0) {
              for (int r = 0; r < 9; ++r) {
                double acc = 0;
                for (int c = 0; c < n1; ++c) acc += Ig[k][c] * T2[(size_t)(i + n1 * (j + n1 * c)) * 9 + r];
                S[r / 3][r % 3] = acc;
              }
            } else {
              cross_rows(G, S);
            }
            for (int d = 0; d < 3; ++d)
              for (int c = 0; c < 3; ++c) put(le, pt * 9 + d * 3 + c, S[d][c]);
            put(le, 9 * nsp + pt, 1 / J);
            for (int c = 0; c < 3; ++c) b.sol_xyz[((size_t)b.canon_pos[le] * nsp + pt) * 3 + c] = x[c];
          }
      // flux points: row d of S on face 2d+s, tangential Gauss coordinates (t0, t1)
      for (int f = 0; f < 6; ++f)
        for (int qq = 0; qq < H.nfpf; ++qq) {
          const int d = f / 2, sd = f % 2, u0 = qq % n1, u1 = qq / n1;
          const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
          const double* L[3];
          const double* D[3];
          L[d] = Lle[sd]; D[d] = dLe[sd];
          L[ta] = Llx[u0]; D[ta] = dLx[u0];
          L[tb] = Llx[u1]; D[tb] = dLx[u1];
          double x[3], G[3][3], row[3];
          geo_at(L[0], D[0], L[1], D[1], L[2], D[2], x, G);
          if (!(det3(G) > 0)) { err = "curved element with J <= 0"; return; }
          if (metric == 0) {
            // the Lobatto end nodes are face values: interpolate along the two tangents only
            const int end = sd ? n1 - 1 : 0;
            for (int c = 0; c < 3; ++c) {
              double acc = 0;
              for (int v1 = 0; v1 < n1; ++v1)
                for (int v0 = 0; v0 < n1; ++v0) {
                  int id[3];
                  id[d] = end; id[ta] = v0; id[tb] = v1;
                  acc += Ig[u0][v0] * Ig[u1][v1] * Ja[(size_t)(id[0] + n1 * (id[1] + n1 * id[2])) * 9 + d * 3 + c];
                }
              row[c] = acc;
            }
          } else {
            double S[3][3];
            cross_rows(G, S);
            for (int c = 0; c < 3; ++c) row[c] = S[d][c];
          }
          const int fp = f * H.nfpf + qq;
          for (int c = 0; c < 3; ++c) put(le, 10 * nsp + fp * 3 + c, row[c]);
        }
    }
  };
  const int64_t nthr = std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                               (b.n + 255) / 256}));
  std::vector<std::string> errs((size_t)nthr);
  std::vector<std::thread> pool;
  for (int64_t t = 0; t < nthr; ++t)
    pool.emplace_back(work, b.n * t / nthr, b.n * (t + 1) / nthr, std::ref(errs[(size_t)t]));
  for (auto& th : pool) th.join();
  for (auto& m : errs)
    if (!m.empty()) { code = 2; return m; }
  // padding lanes copy the first element's terms (in bounds, results discarded)
  for (int r = 0; r < rows; ++r)
    for (int64_t le = b.n; le < b.e_pad; ++le) b.cmet[(size_t)r * b.e_pad + le] = b.cmet[(size_t)r * b.e_pad];
  return "";
}

// ------------------------------------------------------------------ curved tetrahedra
// The same two metrics at the 35 solution points of the order-4 tetrahedron for a map
// of total degree q (1..4) on the equispaced nodes (i, j, k), i + j + k <= q (k
// outermost, then j, then i) at (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q).  Conservative form:
// V^(n) = (x_l - x0_l) grad_xi x_m sampled at the solution points -- they interpolate
// P_4 and 15 of them lie on every face, so the face rows depend only on values the two
// elements of a face share -- and differentiated there with the element's own nodal
// derivative matrices, which are exact for that interpolant.  The flux points are
// solution points, so there is no separate face evaluation.  Stored per solution point
// pt: S (row pt*10 + 3i + j, S_ij = J dxi_i/dx_j) and J (row pt*10 + 9); per flux point fp
// the scaled normal S^T n~ of its face at its collocated point (row 10*nsp + fp*3 + j),
// which the common fluxes use.
std::string build_curved_tet(int q, int metric, const double* xyz, const int64_t* ho, Setup& s, int& code) {
  code = 0;
  Block* bp = nullptr;
  for (auto& b : s.blocks) if (b.etype == kTet) bp = &b;
  if (!bp) { code = 1; return "no tetrahedra"; }
  Block& b = *bp;
  const TetOps& T = s.tet;
  constexpr int N = TetOps::nsp;
  if (q < 1 || q > 4) { code = 3; return "geometry order must be in 1..4"; }
  // geometry nodes and the monomials of total degree <= q (centred at the centroid)
  int lat[N][3], ex[N][3], NQ = 0, NM = 0;
  for (int k = 0; k <= q; ++k)
    for (int j = 0; j <= q - k; ++j)
      for (int i = 0; i <= q - k - j; ++i) { lat[NQ][0] = i; lat[NQ][1] = j; lat[NQ][2] = k; ++NQ; }
  for (int d = 0; d <= q; ++d)
    for (int c = 0; c <= d; ++c)
      for (int bb = 0; bb <= d - c; ++bb) { ex[NM][0] = d - bb - c; ex[NM][1] = bb; ex[NM][2] = c; ++NM; }
  auto mono = [&](const ld* xi, int m, int dir) -> ld {   // monomial m or its derivative along dir (-1: value)
    ld v = 1;
    for (int a = 0; a < 3; ++a) {
      const int e = ex[m][a] - (a == dir ? 1 : 0);
      if (e < 0) return 0;
      ld t = 1;
      for (int r = 0; r < e; ++r) t *= xi[a] + 0.5L;
      v *= (a == dir ? (ld)ex[m][a] : 1) * t;
    }
    return v;
  };
  ld A[N][N];
  for (int n = 0; n < NQ; ++n) {
    ld xi[3];
    for (int a = 0; a < 3; ++a) xi[a] = -1 + 2 * (ld)lat[n][a] / q;
    for (int m = 0; m < NM; ++m) A[n][m] = mono(xi, m, -1);
  }
  if (!invert(A, NQ)) { code = 3; return "singular geometry basis"; }   // l_j = sum_m mono_m A[m][j]
  // basis values and gradients at the solution points
  std::vector<double> Nv((size_t)N * NQ), dN((size_t)N * NQ * 3);
  for (int z = 0; z < N; ++z) {
    ld xi[3] = {T.pts[z][0], T.pts[z][1], T.pts[z][2]};
    for (int j = 0; j < NQ; ++j) {
      ld v = 0, g[3] = {0, 0, 0};
      for (int m = 0; m < NM; ++m) {
        v += mono(xi, m, -1) * A[m][j];
        for (int a = 0; a < 3; ++a) g[a] += mono(xi, m, a) * A[m][j];
      }
      Nv[(size_t)z * NQ + j] = (double)v;
      for (int a = 0; a < 3; ++a) dN[((size_t)z * NQ + j) * 3 + a] = (double)g[a];
    }
  }
  constexpr int NF = TetOps::nfp;
  const int rows = 10 * N + 3 * NF;
  b.cmet.assign((size_t)rows * b.e_pad, 0.0);
  auto work = [&](int64_t lo, int64_t hi, std::string& err) {
    std::vector<double> X((size_t)NQ * 3);
    double x[N][3], G[N][3][3], V[3][N][3];
    for (int64_t le = lo; le < hi; ++le) {
      const int64_t e = b.elems[le];
      for (int n = 0; n < NQ; ++n)
        for (int c = 0; c < 3; ++c) X[(size_t)n * 3 + c] = xyz[ho[e * NQ + n] * 3 + c];
      for (int z = 0; z < N; ++z) {
        for (int c = 0; c < 3; ++c) {
          x[z][c] = 0;
          G[z][c][0] = G[z][c][1] = G[z][c][2] = 0;
        }
        for (int n = 0; n < NQ; ++n) {
          const double w = Nv[(size_t)z * NQ + n];
          const double* d = &dN[((size_t)z * NQ + n) * 3];
          for (int c = 0; c < 3; ++c) {
            x[z][c] += w * X[(size_t)n * 3 + c];
            for (int a = 0; a < 3; ++a) G[z][c][a] += d[a] * X[(size_t)n * 3 + c];
          }
        }
      }
      if (metric == 0)
        for (int z = 0; z < N; ++z)
          for (int n = 0; n < 3; ++n) {
            const int m = (n + 1) % 3, l = (n + 2) % 3;
            for (int k = 0; k < 3; ++k) V[n][z][k] = (x[z][l] - X[l]) * G[z][m][k];
          }
      for (int z = 0; z < N; ++z) {
        const double (&g)[3][3] = G[z];
        const double J = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) - g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0]) +
                         g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
        if (!(J > 0)) { err = "curved element with J <= 0"; return; }
        double S[3][3];
        if (metric == 0) {
          for (int n = 0; n < 3; ++n) {
            double dV[3][3];   // dV[ax][k] = d V^(n)_k / d xi_ax at point z
            for (int ax = 0; ax < 3; ++ax)
              for (int k = 0; k < 3; ++k) {
                double acc = 0;
                for (int y = 0; y < N; ++y) acc += T.D[ax][z][y] * V[n][y][k];
                dV[ax][k] = acc;
              }
            for (int r = 0; r < 3; ++r) {
              const int ra = (r + 1) % 3, rb = (r + 2) % 3;
              S[r][n] = -(dV[ra][rb] - dV[rb][ra]);
            }
          }
        } else {
          // row r = g_{r+1} x g_{r+2}, g_a = column a of G
          for (int r = 0; r < 3; ++r) {
            const int a = (r + 1) % 3, c = (r + 2) % 3;
            S[r][0] = g[1][a] * g[2][c] - g[2][a] * g[1][c];
            S[r][1] = g[2][a] * g[0][c] - g[0][a] * g[2][c];
            S[r][2] = g[0][a] * g[1][c] - g[1][a] * g[0][c];
          }
        }
        for (int r = 0; r < 9; ++r) b.cmet[(size_t)(z * 10 + r) * b.e_pad + le] = S[r / 3][r % 3];
        b.cmet[(size_t)(z * 10 + 9) * b.e_pad + le] = J;
        // S^T n~ at the flux points collocated with this point
        for (int fp = 0; fp < NF; ++fp) {
          if (T.fp_src[fp] != z) continue;
          const double* nr = T.nref[T.fp_face[fp]];
          for (int j = 0; j < 3; ++j)
            b.cmet[(size_t)(10 * N + fp * 3 + j) * b.e_pad + le] = nr[0] * S[0][j] + nr[1] * S[1][j] + nr[2] * S[2][j];
        }
        for (int c = 0; c < 3; ++c) b.sol_xyz[((size_t)b.canon_pos[le] * N + z) * 3 + c] = x[z][c];
      }
    }
  };
  const int64_t nthr = std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                               (b.n + 255) / 256}));
  std::vector<std::string> errs((size_t)nthr);
  std::vector<std::thread> pool;
  for (int64_t t = 0; t < nthr; ++t)
    pool.emplace_back(work, b.n * t / nthr, b.n * (t + 1) / nthr, std::ref(errs[(size_t)t]));
  for (auto& th : pool) th.join();
  for (auto& m : errs)
    if (!m.empty()) { code = 2; return m; }
  for (int r = 0; r < rows; ++r)
    for (int64_t le = b.n; le < b.e_pad; ++le) b.cmet[(size_t)r * b.e_pad + le] = b.cmet[(size_t)r * b.e_pad];
  return "";
}

// ------------------------------------------------------------------ pyramids
// Reference pyramid (kPyrCorner, kPyrFace above): corners (-1,-1,-1) (1,-1,-1) (1,1,-1)
// (-1,1,-1) (0,0,1); faces the base (0 1 2 3) and the triangles (0 1 4) (1 2 4) (2 3 4) (3 0 4).

namespace {
// Basis of the rational space: phi = x^i y^j s^(m-i-j) z^c (= (x/s)^i (y/s)^j s^m z^c),
// m = max(i, j), c <= 4 - m.  At the apex (s = 0) only the m = 0 members are nonzero
// (the others carry s^m with x/s, y/s bounded), which gives their values there.
struct PyrMode { int i, j, m, c; };
std::vector<PyrMode> pyr_modes() {
  std::vector<PyrMode> md;
  for (int i = 0; i <= 4; ++i)
    for (int j = 0; j <= 4; ++j) {
      const int m = std::max(i, j);
      for (int c = 0; c <= 4 - m; ++c) md.push_back({i, j, m, c});
    }
  return md;
}
ld ipow(ld x, int n) { ld r = 1; for (int k = 0; k < n; ++k) r *= x; return r; }
ld pyr_phi(const PyrMode& q, const ld* X) {
  const ld s = (1 - X[2]) / 2;
  if (s < 1e-15L) return q.m == 0 ? ipow(X[2], q.c) : 0;
  const ld a = X[0] / s, b = X[1] / s;
  return ipow(a, q.i) * ipow(b, q.j) * ipow(s, q.m) * ipow(X[2], q.c);
}
// gradient at an interior point: phi = x^i y^j s^e z^c, e = m - i - j, ds/dz = -1/2
void pyr_dphi(const PyrMode& q, const ld* X, ld g[3]) {
  const ld x = X[0], y = X[1], z = X[2], s = (1 - z) / 2;
  const int e = q.m - q.i - q.j;
  const ld se = std::pow(s, (ld)e), zc = ipow(z, q.c);
  const ld xi = ipow(x, q.i), yj = ipow(y, q.j);
  g[0] = q.i ? q.i * ipow(x, q.i - 1) * yj * se * zc : 0;
  g[1] = q.j ? q.j * xi * ipow(y, q.j - 1) * se * zc : 0;
  g[2] = xi * yj * ((e ? -0.5L * e * std::pow(s, (ld)(e - 1)) * zc : 0) + (q.c ? se * q.c * ipow(z, q.c - 1) : 0));
}
}  // namespace

void build_pyr_ops(const TetOps& T, PyrOps& o) {
  constexpr int N = PyrOps::nsp, NF = PyrOps::nfp;
  const std::vector<PyrMode> md = pyr_modes();
  if ((int)md.size() != N) throw std::runtime_error("pyramid space dimension");
  ld g5[5], w5[5];
  gauss_legendre(5, g5, w5);
  // solution points
  int z = 0;
  for (int k = 0; k < 5; ++k) {
    const int n = 5 - k;
    ld g[5], w[5];
    gauss_legendre(n, g, w);
    const ld s = (1 - g5[k]) / 2;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i, ++z) {
        o.pts[z][0] = (double)(s * g[i]);
        o.pts[z][1] = (double)(s * g[j]);
        o.pts[z][2] = (double)g5[k];
      }
  }
  // reference normals
  for (int f = 0; f < 5; ++f) {
    const double* A = kPyrCorner[kPyrFace[f][0]];
    const double* B = kPyrCorner[kPyrFace[f][1]];
    const double* C = kPyrCorner[kPyrFace[f][2]];
    double e1[3], e2[3], nv[3];
    for (int d = 0; d < 3; ++d) { e1[d] = B[d] - A[d]; e2[d] = C[d] - A[d]; }
    cross(e1, e2, nv);
    const double nn = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    double dotc = nv[0] * A[0] + nv[1] * A[1] + nv[2] * (A[2] + 0.5);   // away from the centroid (0,0,-1/2)
    const double sg = dotc > 0 ? 1.0 : -1.0;
    for (int d = 0; d < 3; ++d) o.nref[f][d] = sg * nv[d] / nn;
  }
  // flux points: base grid, then the tetrahedron's face-0 points (corners 0 1 3 of the
  // reference tetrahedron, the plane z = -1: s = (x+1)/2, t = (y+1)/2) on each triangle
  int fp = 0;
  o.face_off[0] = 0;
  for (int j = 0; j < 5; ++j)
    for (int i = 0; i < 5; ++i, ++fp) {
      o.fpts[fp][0] = (double)g5[i]; o.fpts[fp][1] = (double)g5[j]; o.fpts[fp][2] = -1.0;
      o.fp_face[fp] = 0;
    }
  double st[15][2];
  for (int q = 0; q < 15; ++q) {
    const double* X = T.pts[T.fp_src[q]];
    st[q][0] = (X[0] + 1) / 2;
    st[q][1] = (X[1] + 1) / 2;
  }
  for (int f = 1; f < 5; ++f) {
    o.face_off[f] = fp;
    const double* c0 = kPyrCorner[kPyrFace[f][0]];
    const double* c1 = kPyrCorner[kPyrFace[f][1]];
    const double* c2 = kPyrCorner[kPyrFace[f][2]];
    for (int q = 0; q < 15; ++q, ++fp) {
      for (int d = 0; d < 3; ++d) o.fpts[fp][d] = c0[d] + st[q][0] * (c1[d] - c0[d]) + st[q][1] * (c2[d] - c0[d]);
      o.fp_face[fp] = f;
    }
  }
  o.face_off[5] = fp;
  // Lagrange basis l_j = sum_m phi_m C[m][j]
  static ld V[N][N];
  for (int a = 0; a < N; ++a) {
    const ld X[3] = {o.pts[a][0], o.pts[a][1], o.pts[a][2]};
    for (int m = 0; m < N; ++m) V[a][m] = pyr_phi(md[m], X);
  }
  if (!invert(V, N)) throw std::runtime_error("pyramid solution points not unisolvent");
  auto lag = [&](const ld* X, ld* l) {
    ld ph[N];
    for (int m = 0; m < N; ++m) ph[m] = pyr_phi(md[m], X);
    for (int j = 0; j < N; ++j) { ld acc = 0; for (int m = 0; m < N; ++m) acc += ph[m] * V[m][j]; l[j] = acc; }
  };
  for (int f = 0; f < NF; ++f) {
    const ld X[3] = {o.fpts[f][0], o.fpts[f][1], o.fpts[f][2]};
    ld l[N];
    lag(X, l);
    for (int j = 0; j < N; ++j) o.interp[f][j] = (double)l[j];
  }
  for (int a = 0; a < N; ++a) {
    const ld X[3] = {o.pts[a][0], o.pts[a][1], o.pts[a][2]};
    ld dp[N][3];
    for (int m = 0; m < N; ++m) pyr_dphi(md[m], X, dp[m]);
    for (int d = 0; d < 3; ++d)
      for (int j = 0; j < N; ++j) {
        ld acc = 0;
        for (int m = 0; m < N; ++m) acc += dp[m][d] * V[m][j];
        o.D[d][a][j] = (double)acc;
      }
  }
  // mass matrix by the collapsed Gauss rule x = s a, y = s b, dV = s^2 da db dz (8 points
  // per direction: exact for the degree-(8, 8, 10) integrands in (a, b, z))
  ld g8[8], w8[8];
  gauss_legendre(8, g8, w8);
  static ld M[N][N];
  for (int i = 0; i < N; ++i) for (int j = 0; j < N; ++j) M[i][j] = 0;
  for (int ka = 0; ka < 8; ++ka)
    for (int kb = 0; kb < 8; ++kb)
      for (int kz = 0; kz < 8; ++kz) {
        const ld s = (1 - g8[kz]) / 2;
        const ld X[3] = {s * g8[ka], s * g8[kb], g8[kz]};
        const ld w = w8[ka] * w8[kb] * w8[kz] * s * s;
        ld l[N];
        lag(X, l);
        for (int i = 0; i < N; ++i) for (int j = 0; j < N; ++j) M[i][j] += w * l[i] * l[j];
      }
  if (!invert(M, N)) throw std::runtime_error("pyramid mass matrix singular");
  // face matrices E[i][sigma] = int_face l_i phi_sigma dS (true face areas)
  static ld Em[N][NF];
  for (int i = 0; i < N; ++i) for (int f = 0; f < NF; ++f) Em[i][f] = 0;
  ld g7[7], w7[7];
  gauss_legendre(7, g7, w7);
  for (int qa = 0; qa < 7; ++qa)                       // base: tensor Lagrange on the 5 x 5 grid, dS = dx dy
    for (int qb = 0; qb < 7; ++qb) {
      const ld X[3] = {g7[qa], g7[qb], -1};
      ld l[N], lx[5], ly[5], dd[5];
      lag(X, l);
      lagrange_1d(g5, 5, g7[qa], lx, dd);
      lagrange_1d(g5, 5, g7[qb], ly, dd);
      const ld w = w7[qa] * w7[qb];
      for (int i = 0; i < N; ++i)
        for (int jj = 0; jj < 5; ++jj)
          for (int ii = 0; ii < 5; ++ii) Em[i][jj * 5 + ii] += w * l[i] * lx[ii] * ly[jj];
    }
  // triangles: Lagrange of total degree 4 on the 15 face points (monomials s^a t^b)
  static ld Q[15][15];
  auto tmono = [](ld s_, ld t_, ld* out) {
    int k = 0;
    for (int d = 0; d <= 4; ++d) for (int a = 0; a <= d; ++a) out[k++] = ipow(s_, a) * ipow(t_, d - a);
  };
  for (int q = 0; q < 15; ++q) tmono(st[q][0], st[q][1], Q[q]);
  if (!invert(Q, 15)) throw std::runtime_error("triangle face points not unisolvent");
  for (int f = 1; f < 5; ++f) {
    const double* c0 = kPyrCorner[kPyrFace[f][0]];
    const double* c1 = kPyrCorner[kPyrFace[f][1]];
    const double* c2 = kPyrCorner[kPyrFace[f][2]];
    double e1[3], e2[3], cr[3];
    for (int d = 0; d < 3; ++d) { e1[d] = c1[d] - c0[d]; e2[d] = c2[d] - c0[d]; }
    cross(e1, e2, cr);
    const ld jac = std::sqrt((ld)cr[0] * cr[0] + (ld)cr[1] * cr[1] + (ld)cr[2] * cr[2]);   // 2 x area
    for (int qa = 0; qa < 7; ++qa)                     // collapsed rule on the unit triangle
      for (int qb = 0; qb < 7; ++qb) {
        const ld t_ = (g7[qb] + 1) / 2, s_ = (g7[qa] + 1) / 2 * (1 - t_);
        const ld w = w7[qa] * w7[qb] / 4 * (1 - t_) * jac;
        ld X[3];
        for (int d = 0; d < 3; ++d) X[d] = c0[d] + s_ * e1[d] + t_ * e2[d];
        ld l[N], mo[15];
        lag(X, l);
        tmono(s_, t_, mo);
        for (int q = 0; q < 15; ++q) {
          ld phi = 0;
          for (int k = 0; k < 15; ++k) phi += mo[k] * Q[k][q];
          for (int i = 0; i < N; ++i) Em[i][o.face_off[f] + q] += w * l[i] * phi;
        }
      }
  }
  for (int i = 0; i < N; ++i)
    for (int f = 0; f < NF; ++f) {
      ld acc = 0;
      for (int k = 0; k < N; ++k) acc += M[i][k] * Em[k][f];
      o.lift[i][f] = (double)acc;
    }
}

}  // namespace frmi
