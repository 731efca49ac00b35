// Host-side 1D rules and operator tables of the gfx950 library, computed in long double
// and rounded once.  (Section "Nodal bases, quadrature, and mass matrices" and
// eq. euler-sbp.)
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

typedef long double ld;

// Legendre P_n and P_n' at x (three-term recurrence; derivative from the recurrence of
// derivatives, valid at the end points too).
static void leg(int n, ld x, ld* P, ld* dP) {
  ld p0 = 1, p1 = x, d0 = 0, d1 = 1;
  if (n == 0) { *P = 1; *dP = 0; return; }
  for (int k = 1; k < n; ++k) {
    ld p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    ld d2 = d0 + (2 * k + 1) * p1;  // P'_{k+1} = P'_{k-1} + (2k+1) P_k
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1; *dP = d1;
}

static std::vector<ld> gauss_nodes(int npts, std::vector<ld>& w) {
  std::vector<ld> x(npts);
  w.assign(npts, 0);
  for (int k = 0; k < npts; ++k) {
    ld z = std::cos((ld)M_PI * (npts - k - 0.25L) / (npts + 0.5L));
    for (int it = 0; it < 60; ++it) {
      ld P, dP; leg(npts, z, &P, &dP);
      ld dz = P / dP; z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    ld P, dP; leg(npts, z, &P, &dP);
    x[k] = z; w[k] = 2 / ((1 - z * z) * dP * dP);
  }
  return x;
}

static std::vector<ld> gll_nodes(int r, std::vector<ld>& w) {
  std::vector<ld> x(r + 1);
  w.assign(r + 1, 0);
  if (r == 0) { x[0] = 0; w[0] = 2; return x; }
  x[0] = -1; x[r] = 1;
  for (int k = 1; k < r; ++k) {
    ld z = -std::cos((ld)M_PI * k / r);
    for (int it = 0; it < 60; ++it) {
      // roots of P_r': Newton on q = P_r' with q' from Legendre's equation
      ld P, dP; leg(r, z, &P, &dP);
      ld d2 = (2 * z * dP - r * (r + 1) * P) / (1 - z * z);
      ld dz = dP / d2; z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    x[k] = z;
  }
  for (int k = 0; k <= r; ++k) { ld P, dP; leg(r, x[k], &P, &dP); w[k] = 2 / (r * (r + 1) * P * P); }
  return x;
}

// value and derivative of Lagrange basis s of node set xs at point t
static ld lag_val(const std::vector<ld>& xs, int s, ld t) {
  ld v = 1;
  for (size_t k = 0; k < xs.size(); ++k) if ((int)k != s) v *= (t - xs[k]) / (xs[s] - xs[k]);
  return v;
}
static ld lag_der(const std::vector<ld>& xs, int s, ld t) {
  ld sum = 0;
  for (size_t l = 0; l < xs.size(); ++l) {
    if ((int)l == s) continue;
    ld prod = 1 / (xs[s] - xs[l]);
    for (size_t k = 0; k < xs.size(); ++k)
      if ((int)k != s && k != l) prod *= (t - xs[k]) / (xs[s] - xs[k]);
    sum += prod;
  }
  return sum;
}

static void fill(double (*M)[MHD_MAXN], const std::vector<ld>& src, const std::vector<ld>& dst, bool der) {
  for (size_t t = 0; t < dst.size(); ++t)
    for (size_t s = 0; s < src.size(); ++s)
      M[t][s] = (double)(der ? lag_der(src, (int)s, dst[t]) : lag_val(src, (int)s, dst[t]));
}

void build_hydro_tables(int p, HydroTab* T) {
  std::memset(T, 0, sizeof(*T));
  std::vector<ld> w, x = gll_nodes(p, w);
  const int n = p + 1;
  std::vector<ld> D(n * n);
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < n; ++r) D[i * n + r] = lag_der(x, r, x[i]);
  for (int i = 0; i < n; ++i) { T->xi[i] = (double)x[i]; T->w[i] = (double)w[i]; }
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < n; ++r) {
      ld S = w[i] * D[i * n + r] - w[r] * D[r * n + i];  // Q - Q^T
      T->Shat[i][r] = (double)(S / w[i]);
    }
  for (int a = 0; a < n; ++a) {
    ld nrm = 0;
    for (int i = 0; i < n; ++i) { ld P, dP; leg(a, x[i], &P, &dP); nrm += w[i] * P * P; T->V[i][a] = (double)P; }
    for (int i = 0; i < n; ++i) { ld P, dP; leg(a, x[i], &P, &dP); T->Tf[a][i] = (double)(w[i] * P / nrm); }
  }
  // derivative end rows from powers of D (exact on P_p)
  std::vector<ld> Dr(n * n, 0), tmp(n * n);
  for (int i = 0; i < n; ++i) Dr[i * n + i] = 1;
  for (int r = 0; r < n; ++r) {
    for (int i = 0; i < n; ++i) { T->Dr0[r][i] = (double)Dr[0 * n + i]; T->Drp[r][i] = (double)Dr[(n - 1) * n + i]; }
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        ld s = 0;
        for (int k = 0; k < n; ++k) s += D[a * n + k] * Dr[k * n + b];
        tmp[a * n + b] = s;
      }
    Dr = tmp;
  }
  int k = 0;
  for (int l = 0; l < n; ++l)
    for (int a = 0; a <= l; ++a)
      for (int b = 0; b <= l; ++b)
        if (a == l || b == l) { T->ka[k] = a; T->kb[k] = b; T->ksh[k] = l; ++k; }
  ld f = 1;
  for (int r = 0; r < n; ++r) {
    if (r > 0) f *= r;
    T->fr[r] = (double)((2 * r + 1) * std::pow((ld)2, r) / (2 * f));
  }
}

void build_mag_tables(int p, int m, MagTab* T) {
  std::memset(T, 0, sizeof(*T));
  std::vector<ld> ww, wg, wq, wv, wp;
  std::vector<ld> xw = gll_nodes(m + 1, ww), xg = gauss_nodes(m + 1, wg), xq = gauss_nodes(m + 2, wq);
  std::vector<ld> xv = gll_nodes(m, wv), xp = gll_nodes(p, wp);
  for (size_t k = 0; k < xw.size(); ++k) { T->xw[k] = (double)xw[k]; T->ww[k] = (double)ww[k]; }
  for (size_t k = 0; k < xg.size(); ++k) { T->xg[k] = (double)xg[k]; T->wg[k] = (double)wg[k]; }
  for (size_t k = 0; k < xq.size(); ++k) { T->xq[k] = (double)xq[k]; T->wq[k] = (double)wq[k]; }
  for (size_t k = 0; k < xv.size(); ++k) { T->xv[k] = (double)xv[k]; T->wv[k] = (double)wv[k]; }
  for (size_t k = 0; k < xp.size(); ++k) { T->xp[k] = (double)xp[k]; T->wp[k] = (double)wp[k]; }
  fill(T->I_W_Q, xw, xq, false); fill(T->D_W_Q, xw, xq, true); fill(T->I_G_Q, xg, xq, false);
  fill(T->D_W_G, xw, xg, true); fill(T->I_V_G, xv, xg, false);
  fill(T->I_P_G, xp, xg, false); fill(T->I_P_W, xp, xw, false);
  fill(T->I_W_G, xw, xg, false); fill(T->I_G_W, xg, xw, false); fill(T->I_V_W, xv, xw, false);
  fill(T->I_G_P, xg, xp, false); fill(T->I_W_P, xw, xp, false); fill(T->I_V_P, xv, xp, false);
  fill(T->D_W_V, xw, xv, true); fill(T->I_G_V, xg, xv, false);
  fill(T->I_V_Q, xv, xq, false);
  std::vector<ld> ends = {-1, 1};
  for (int s = 0; s < 2; ++s) {
    for (size_t k = 0; k < xg.size(); ++k) T->I_G_E[s][k] = (double)lag_val(xg, (int)k, ends[s]);
    for (size_t k = 0; k < xv.size(); ++k) T->I_V_E[s][k] = (double)lag_val(xv, (int)k, ends[s]);
  }
}
