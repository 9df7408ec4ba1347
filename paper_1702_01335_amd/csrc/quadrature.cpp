// Host-side quadrature and Hermite projection tables for the mixed half-range /
// full-range lattice Boltzmann velocity set (Ambrus & Sofonea, arXiv:1702.01335, Sec. III).
//
// x axis: half-range Gauss-Hermite rule with Qx nodes per semi-axis for the weight
//   omega(p) = exp(-p^2/2)/sqrt(2 pi) on [0, inf) (the rule recovers half-space moments up
//   to order 2Qx-1).  Its recurrence coefficients come from the discretised Stieltjes
//   procedure on a composite Gauss-Legendre discretisation of [0, 40] in long double;
//   nodes from the Jacobi matrix (Sturm-sequence bisection), Newton-polished on the
//   recurrence;
//   weights from the Christoffel sum, which keeps relative accuracy for tiny weights.
// y, z axes: full-range rule for the same omega on R (probabilists' Hermite He_l,
//   recurrence He_{l+1} = p He_l - l He_{l-1}).
// Projection tables (Sec. III direct-product construction): for the x semi-axis
//   phi[m][l] = w_m h_l(p_m) / gamma_l and the monomial coefficients of the monic h_l;
//   for y, z phi[j][l] = w_j He_l(p_j) / l!.
#include "hrlb_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace hrlb {

typedef long double ld;

static const ld PI_L = 3.141592653589793238462643383279502884L;

// Gauss-Legendre nodes/weights on [-1, 1] in long double (Newton on the Legendre recurrence).
static void gauss_legendre(int m, std::vector<ld>& x, std::vector<ld>& w) {
  x.assign(m, 0.0L);
  w.assign(m, 0.0L);
  for (int i = 0; i < (m + 1) / 2; ++i) {
    ld z = std::cos(PI_L * (i + 0.75L) / (m + 0.5L));
    ld dp = 0;
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= m; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = m * (z * p1 - p0) / (z * z - 1);
      ld dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-21L) break;
    }
    ld p0 = 1, p1 = z;
    for (int k = 2; k <= m; ++k) {
      ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = m * (z * p1 - p0) / (z * z - 1);
    x[i] = -z;
    x[m - 1 - i] = z;
    w[i] = w[m - 1 - i] = 2 / ((1 - z * z) * dp * dp);
  }
}

// Recurrence coefficients (a_k, b_k), k <= n, of the monic polynomials orthogonal to
// exp(-p^2/2)/sqrt(2 pi) on [0, inf), by the discretised Stieltjes procedure.
static void half_range_recurrence(int n, std::vector<ld>& a, std::vector<ld>& b) {
  const ld P = 40.0L, h = 0.5L;
  const int panels = (int)(P / h);
  const int m = std::min(n + 48, 400);
  std::vector<ld> gx, gw;
  gauss_legendre(m, gx, gw);
  std::vector<ld> X, W;
  X.reserve((size_t)panels * m);
  W.reserve((size_t)panels * m);
  const ld c = 1.0L / std::sqrt(2 * PI_L);
  for (int pnl = 0; pnl < panels; ++pnl) {
    ld lo = pnl * h;
    for (int i = 0; i < m; ++i) {
      ld xx = lo + h * (gx[i] + 1) / 2;
      X.push_back(xx);
      W.push_back(gw[i] * h / 2 * c * std::exp(-xx * xx / 2));
    }
  }
  const size_t M = X.size();
  std::vector<ld> pm1(M, 0.0L), p0(M, 1.0L), p1(M);
  a.assign(n + 1, 0.0L);
  b.assign(n + 1, 0.0L);
  ld norm_prev = 1;
  for (int k = 0; k <= n; ++k) {
    ld nrm = 0, xn = 0;
    for (size_t i = 0; i < M; ++i) {
      ld t = W[i] * p0[i] * p0[i];
      nrm += t;
      xn += t * X[i];
    }
    a[k] = xn / nrm;
    b[k] = (k == 0) ? nrm : nrm / norm_prev;
    norm_prev = nrm;
    for (size_t i = 0; i < M; ++i) p1[i] = (X[i] - a[k]) * p0[i] - b[k] * pm1[i];
    pm1.swap(p0);
    p0.swap(p1);
  }
}

// Eigenvalues of the symmetric tridiagonal (Jacobi) matrix with diagonal d and
// off-diagonal e[1..n-1], by bisection on Sturm sequence counts: the number of negative
// pivots of the LDL^T factorisation of J - x I is the number of eigenvalues below x.
static int count_below(const std::vector<ld>& d, const std::vector<ld>& e, ld x) {
  int cnt = 0;
  ld q = 1;
  for (size_t i = 0; i < d.size(); ++i) {
    ld off = (i == 0) ? 0.0L : e[i] * e[i] / q;
    q = d[i] - x - off;
    if (q == 0) q = -1e-4000L;
    if (q < 0) ++cnt;
  }
  return cnt;
}

static void tridiag_eigenvalues(const std::vector<ld>& d, const std::vector<ld>& e, std::vector<ld>& out) {
  const int n = (int)d.size();
  ld lo = d[0], hi = d[0];
  for (int i = 0; i < n; ++i) {  // Gershgorin interval
    ld r = (i > 0 ? std::fabs(e[i]) : 0.0L) + (i + 1 < n ? std::fabs(e[i + 1]) : 0.0L);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  out.assign(n, 0.0L);
  for (int k = 0; k < n; ++k) {
    ld a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 1e-19L * (std::fabs(a) + std::fabs(b)); ++it) {
      ld mid = (a + b) / 2;
      if (count_below(d, e, mid) > k)
        b = mid;
      else
        a = mid;
    }
    out[k] = (a + b) / 2;
  }
}

// Gauss rule with Q nodes from the recurrence (a, b): nodes = zeros of P_Q, weights =
// 1 / sum_{k<Q} P_k(x)^2 / (b_0 ... b_k).
static void gauss_from_recurrence(int Q, const std::vector<ld>& a, const std::vector<ld>& b,
                                  std::vector<ld>& x, std::vector<ld>& w) {
  std::vector<ld> d(a.begin(), a.begin() + Q), e(Q, 0.0L);
  for (int k = 1; k < Q; ++k) e[k] = std::sqrt(b[k]);
  tridiag_eigenvalues(d, e, x);
  w.assign(Q, 0.0L);
  for (int i = 0; i < Q; ++i) {
    ld z = x[i];
    for (int it = 0; it < 50; ++it) {
      ld p0 = 1, p1 = z - a[0], d0 = 0, d1 = 1;
      for (int k = 1; k < Q; ++k) {
        ld p2 = (z - a[k]) * p1 - b[k] * p0;
        ld d2 = p1 + (z - a[k]) * d1 - b[k] * d0;
        p0 = p1;
        p1 = p2;
        d0 = d1;
        d1 = d2;
      }
      if (Q == 1) {
        p1 = z - a[0];
        d1 = 1;
      }
      ld dz = p1 / d1;
      z -= dz;
      if (std::fabs(dz) <= 1e-20L * (std::fabs(z) + 1e-3L)) break;
    }
    x[i] = z;
    ld norm = b[0], pk = 1, pkm1 = 0, sum = 1 / norm;
    for (int k = 1; k < Q; ++k) {
      ld pn = (z - a[k - 1]) * pk - (k >= 2 ? b[k - 1] : 0.0L) * pkm1;
      pkm1 = pk;
      pk = pn;
      norm *= b[k];
      sum += pk * pk / norm;
    }
    w[i] = 1 / sum;
  }
}

int build_quadrature(int Qx, int Nx, int Qy, int Ny, int Qz, int Nz, QuadTables& qt) {
  qt.Qx = Qx;
  qt.Nx = Nx;
  qt.Qy = Qy;
  qt.Ny = Ny;
  qt.Qz = Qz;
  qt.Nz = Nz;
  qt.reduced = 0;
  // ---- x axis ----
  std::vector<ld> a, b, xh, wh;
  half_range_recurrence(Qx + 1, a, b);
  gauss_from_recurrence(Qx, a, b, xh, wh);
  qt.px.assign(2 * Qx, 0.0);
  qt.wx.assign(2 * Qx, 0.0);
  for (int m = 0; m < Qx; ++m) {
    qt.px[Qx + m] = (double)xh[m];
    qt.px[Qx - 1 - m] = -(double)xh[m];
    qt.wx[Qx + m] = qt.wx[Qx - 1 - m] = (double)wh[m];
  }
  // monic h_l coefficients and norms gamma_l = b_0 ... b_l
  std::vector<std::vector<ld>> C(Nx + 1, std::vector<ld>(Nx + 1, 0.0L));
  C[0][0] = 1;
  if (Nx >= 1) {
    C[1][0] = -a[0];
    C[1][1] = 1;
  }
  for (int l = 1; l < Nx; ++l)
    for (int k = 0; k <= Nx; ++k)
      C[l + 1][k] = (k > 0 ? C[l][k - 1] : 0.0L) - a[l] * C[l][k] - b[l] * C[l - 1][k];
  std::vector<ld> gam(Nx + 1);
  gam[0] = b[0];
  for (int l = 1; l <= Nx; ++l) gam[l] = gam[l - 1] * b[l];
  qt.cx.assign((size_t)(Nx + 1) * (Nx + 1), 0.0);
  for (int l = 0; l <= Nx; ++l)
    for (int k = 0; k <= Nx; ++k) qt.cx[l * (Nx + 1) + k] = (double)C[l][k];
  qt.phix.assign((size_t)Qx * (Nx + 1), 0.0);
  for (int m = 0; m < Qx; ++m) {
    ld z = xh[m], pk = 1, pkm1 = 0;
    for (int l = 0; l <= Nx; ++l) {
      if (l > 0) {
        ld pn = (z - a[l - 1]) * pk - (l >= 2 ? b[l - 1] : 0.0L) * pkm1;
        pkm1 = pk;
        pk = pn;
      }
      qt.phix[m * (Nx + 1) + l] = (double)(wh[m] * pk / gam[l]);
    }
  }
  // ---- y, z axes ----
  auto full = [](int Q, int N, std::vector<double>& p, std::vector<double>& w, std::vector<double>& phi) {
    std::vector<ld> fa(Q + 1, 0.0L), fb(Q + 1);
    fb[0] = 1;
    for (int k = 1; k <= Q; ++k) fb[k] = k;
    std::vector<ld> xx, ww;
    gauss_from_recurrence(Q, fa, fb, xx, ww);
    p.assign(Q, 0.0);
    w.assign(Q, 0.0);
    for (int j = 0; j < Q; ++j) {
      // bitwise symmetry: p_{Q-1-j} = -p_j, equal weights
      ld pj = (xx[j] - xx[Q - 1 - j]) / 2, wj = (ww[j] + ww[Q - 1 - j]) / 2;
      p[j] = (double)pj;
      w[j] = (double)wj;
    }
    phi.assign((size_t)Q * (N + 1), 0.0);
    for (int j = 0; j < Q; ++j) {
      ld z = p[j], hk = 1, hkm1 = 0, fact = 1;
      for (int l = 0; l <= N; ++l) {
        if (l > 0) {
          ld hn = z * hk - (l - 1) * hkm1;
          hkm1 = hk;
          hk = hn;
          fact *= l;
        }
        phi[j * (N + 1) + l] = (double)((ld)w[j] * hk / fact);
      }
    }
  };
  full(Qy, Ny, qt.py, qt.wy, qt.phiy);
  full(Qz, Nz, qt.pz, qt.wz, qt.phiz);
  return 0;
}

}  // namespace hrlb
