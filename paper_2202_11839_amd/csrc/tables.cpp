// Host tables of a plan: output series, the list of FFT fields with their
// line-of-sight weight polynomials, and the integer k-shell thresholds.
#include <cmath>
#include <cstdio>

#include "lpp_internal.h"

namespace lpp {

namespace {

double factorial(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

double binomial(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  return factorial(n) / (factorial(k) * factorial(n - k));
}

// Power-basis coefficients of the Legendre polynomial L_L(z):
// L_L(z) = 2^-L sum_k (-1)^k C(L,k) C(2L-2k, L) z^(L-2k)  (exact in double for L <= 8).
std::vector<double> legendre_coefs(int L) {
  std::vector<double> c(L + 1, 0.0);
  for (int k = 0; 2 * k <= L; ++k) {
    double v = binomial(L, k) * binomial(2 * L - 2 * k, L) / std::ldexp(1.0, L);
    c[L - 2 * k] = (k % 2 ? -v : v);
  }
  return c;
}

std::vector<double> derivative(const std::vector<double>& c, int times) {
  std::vector<double> d = c;
  for (int t = 0; t < times; ++t) {
    if (d.size() <= 1) return {0.0};
    std::vector<double> e(d.size() - 1);
    for (size_t i = 1; i < d.size(); ++i) e[i - 1] = d[i] * static_cast<double>(i);
    d.swap(e);
  }
  return d;
}

}  // namespace

double prefactor(int m, int L) { return (2 * L + 1) * factorial(L - m) / factorial(L + m); }

// C_{lL} = (2l+1) int_{-1}^{1} dmu/2 L^4_L(mu) L_l(mu), with
// L^4_L = (1-mu^2)^2 d^4 L_L/dmu^4 (Condon-Shortley sign (+1) for m = 4).
double cmap_minus_to_legendre(int l, int L) {
  std::vector<double> r = derivative(legendre_coefs(L), 4);
  std::vector<double> w = {1.0, 0.0, -2.0, 0.0, 1.0};  // (1-mu^2)^2
  std::vector<double> ll = legendre_coefs(l);
  std::vector<double> p(r.size() + w.size() + ll.size(), 0.0);
  for (size_t i = 0; i < r.size(); ++i)
    for (size_t j = 0; j < w.size(); ++j)
      for (size_t k = 0; k < ll.size(); ++k) p[i + j + k] += r[i] * w[j] * ll[k];
  double s = 0.0;
  for (size_t i = 0; i < p.size(); i += 2) s += p[i] / static_cast<double>(i + 1);
  return (2 * l + 1) * s;
}

FieldSpec make_spec(int s, int L, int M, int cs) {
  FieldSpec f{};
  f.s = s;
  f.L = L;
  f.M = M;
  f.cs = cs;
  std::vector<double> leg = legendre_coefs(L);
  for (int j = 0; j <= s; ++j) {
    std::vector<double> d = derivative(leg, M + j);
    double fac = (j % 2 ? -1.0 : 1.0) / factorial(j);
    f.nq[j] = static_cast<int32_t>(d.size());
    for (size_t i = 0; i < d.size() && i < 9; ++i) f.q[j][i] = d[i] * fac;
    f.binom[j] = binomial(M, s - j);
  }
  double kappa = (M == 0) ? 1.0 : 2.0 * factorial(L - M) / factorial(L + M);
  f.scale = kappa * factorial(s);
  return f;
}

bool build_tables(const lpp_config& cfg, Tables& t) {
  t = Tables{};
  const int lmax = cfg.lmax;
  const uint32_t sp = cfg.spectra;
  auto add = [&](const std::string& name, int fam, int L) {
    t.series_of_acc.push_back(static_cast<int>(t.series.size()));
    t.series.push_back(name);
    t.acc_series.push_back(fam);
    t.acc_L.push_back(L);
  };
  char buf[32];
  if (sp & LPP_DD)
    for (int l = 0; l <= lmax; l += 2) {
      std::snprintf(buf, sizeof buf, "DD_l%d", l);
      if (l == 0) t.dd0 = static_cast<int>(t.acc_series.size());
      add(buf, FAM_DD, l);
    }
  if (sp & LPP_GD)
    for (int L = 2; L <= lmax; L += 2) {
      std::snprintf(buf, sizeof buf, "GD_L%d", L);
      add(buf, FAM_GD, L);
    }
  if (sp & LPP_PLUS)
    for (int l = 0; l <= lmax; l += 2) {
      std::snprintf(buf, sizeof buf, "PLUS_l%d", l);
      if (l == 0) t.plus0 = static_cast<int>(t.acc_series.size());
      add(buf, FAM_PLUS, l);
    }
  if (sp & LPP_MINUS)
    for (int L = 4; L <= lmax; L += 2) {
      std::snprintf(buf, sizeof buf, "MINUS_L%d", L);
      add(buf, FAM_MINUS, L);
    }
  if ((sp & LPP_PLUS) && (sp & LPP_MINUS) && lmax >= 4) {
    for (int l = 0; l <= lmax; l += 2) {
      std::snprintf(buf, sizeof buf, "EE_l%d", l);
      t.series.push_back(buf);
    }
    for (int l = 0; l <= lmax; l += 2) {
      std::snprintf(buf, sizeof buf, "BB_l%d", l);
      t.series.push_back(buf);
    }
  }
  // fields with L > 0, grouped by accumulator series
  for (size_t a = 0; a < t.acc_series.size(); ++a) {
    const int fam = t.acc_series[a];
    const int L = t.acc_L[a];
    if (L == 0) continue;  // the monopoles come from the bases
    const int s = (fam == FAM_GD) ? 2 : (fam == FAM_MINUS ? 4 : 0);
    for (int M = 0; M <= L; ++M)
      for (int cs = 0; cs < (M == 0 ? 1 : 2); ++cs) {
        Field f;
        f.fam = static_cast<Family>(fam);
        f.series = static_cast<int>(a);
        f.spec = make_spec(s, L, M, cs);
        t.fields.push_back(f);
      }
  }
  // thresholds T_b = ceil((b num/den)^2), exact in 64-bit integers
  int64_t num = cfg.dn_num, den = cfg.dn_den;
  t.thr.resize(cfg.n_kbins + 1);
  for (int b = 0; b <= cfg.n_kbins; ++b) {
    const int64_t a = static_cast<int64_t>(b) * num;
    const int64_t q = a * a, d2 = den * den;
    t.thr[b] = (q + d2 - 1) / d2;
  }
  return true;
}

}  // namespace lpp
