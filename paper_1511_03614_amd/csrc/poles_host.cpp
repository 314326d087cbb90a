// Sectors with monomial exponents a_j < -1 (a propagator power above one, or
// d0 below 4, after decomposition; eq. (2)), reduced on the host to sectors
// with a_j >= -1, which the evaluator's subtraction handles.
//
// The integral over x_j is the analytic continuation in eps.  With
// alpha = a_j + 1 + b_j eps, x^(a_j + b_j eps) = (1/alpha) d/dx x^alpha, and
// integrating by parts (the boundary term at 0 vanishes in the continuation)
//   int_0^1 x^(a+b eps) G dx = G|_(x_j = 1) / alpha - (1/alpha) int_0^1 x^alpha dG/dx_j dx,
//   dG/dx_j = sum_m (g_m + d_m eps) (dP_m/dx_j) P_m^(g_m - 1 + d_m eps) prod_(m' != m) P_m'^(...).
// Each step raises a_j by one.  The parts carry coefficient series in eps
// (1/alpha, (g_m + d_m eps)) that multiply the prefactor in the fold.
//
// Order (the same as the reference implementation's): input sectors in
// order; within one, the lowest variable with a_j < -1 first, the boundary
// part (x_j = 1: x_j's exponents set to 0, equal rows merged in order of first
// occurrence, a_j = b_j = 0) before the derivative parts by factor index,
// depth first; a factor whose exponent becomes (0, 0) is dropped, the
// derivative factor (exponent (1, 0), terms in P_m's order) appended last.
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "host.h"
#include "poles.h"

namespace sdi {

namespace {

using cplx = std::complex<double>;

struct Fac {
  double g, d;
  std::vector<double> coef;
  std::vector<uint8_t> exps;   // [terms][n]
};

struct Sec {
  int n;
  std::vector<double> a, b;
  std::vector<Fac> f;
  std::vector<cplx> series;
  double cre, cim;
};

std::vector<cplx> mul(const std::vector<cplx>& s, const std::vector<cplx>& t) {
  std::vector<cplx> o(POLE_SERIES_LEN, 0.0);
  for (int i = 0; i < POLE_SERIES_LEN; ++i)
    for (int j = 0; i + j < POLE_SERIES_LEN && j < (int)t.size(); ++j) o[i + j] += s[i] * t[j];
  return o;
}

Fac at_one(const Fac& f, int n, int j) {
  Fac o{f.g, f.d, {}, {}};
  std::map<std::vector<uint8_t>, size_t> at;
  const size_t T = f.coef.size();
  for (size_t t = 0; t < T; ++t) {
    std::vector<uint8_t> e(f.exps.begin() + t * n, f.exps.begin() + (t + 1) * n);
    e[j] = 0;
    auto it = at.find(e);
    if (it == at.end()) {
      at.emplace(e, o.coef.size());
      o.coef.push_back(f.coef[t]);
      o.exps.insert(o.exps.end(), e.begin(), e.end());
    } else {
      o.coef[it->second] += f.coef[t];
    }
  }
  Fac k{f.g, f.d, {}, {}};
  for (size_t t = 0; t < o.coef.size(); ++t)
    if (o.coef[t] != 0.0) {
      k.coef.push_back(o.coef[t]);
      k.exps.insert(k.exps.end(), o.exps.begin() + t * n, o.exps.begin() + (t + 1) * n);
    }
  return k;
}

bool derivative(const Fac& f, int n, int j, Fac& out) {
  out = Fac{1.0, 0.0, {}, {}};
  for (size_t t = 0; t < f.coef.size(); ++t) {
    const uint8_t ej = f.exps[t * n + j];
    if (ej == 0) continue;
    out.coef.push_back(f.coef[t] * (double)ej);
    for (int q = 0; q < n; ++q) out.exps.push_back(q == j ? (uint8_t)(ej - 1) : f.exps[t * n + q]);
  }
  return !out.coef.empty();
}

int expand(const Sec& s, std::vector<Sec>& out, int depth, std::string& err) {
  int j = -1;
  for (int q = 0; q < s.n && j < 0; ++q)
    if (s.a[q] < -1.0) j = q;
  if (j < 0) {
    out.push_back(s);
    return SDI_OK;
  }
  if (depth > 16 || out.size() > 100000) {
    err = "expansion of a_j < -1 grew too large";
    return SDI_ENOTSUP;
  }
  const double a0 = s.a[j] + 1.0, b = s.b[j];
  if (b == 0.0) {
    err = "a_j < -1 needs b_j != 0";
    return SDI_EINVAL;
  }
  std::vector<cplx> inv(POLE_SERIES_LEN), minv(POLE_SERIES_LEN);
  for (int q = 0; q < POLE_SERIES_LEN; ++q) {
    inv[q] = (1.0 / a0) * std::pow(-b / a0, q);
    minv[q] = -inv[q];
  }
  // boundary part, x_j = 1
  {
    Sec B{s.n, s.a, s.b, {}, mul(s.series, inv), s.cre, s.cim};
    B.a[j] = 0.0;
    B.b[j] = 0.0;
    bool zero = false;
    for (const Fac& f : s.f) {
      Fac g = at_one(f, s.n, j);
      if (g.coef.empty()) {
        if (!(f.g > 0.0)) {
          err = "a factor vanishes at x_j = 1 with a non-positive exponent";
          return SDI_EINVAL;
        }
        zero = true;
      }
      B.f.push_back(std::move(g));
    }
    if (!zero) {
      const int rc = expand(B, out, depth + 1, err);
      if (rc != SDI_OK) return rc;
    }
  }
  // derivative parts
  for (size_t m = 0; m < s.f.size(); ++m) {
    Fac D;
    if (!derivative(s.f[m], s.n, j, D)) continue;
    Sec C{s.n, s.a, s.b, {}, mul(mul(s.series, minv), {cplx(s.f[m].g), cplx(s.f[m].d)}), s.cre, s.cim};
    C.a[j] += 1.0;
    for (size_t mm = 0; mm < s.f.size(); ++mm) {
      if (mm != m) {
        C.f.push_back(s.f[mm]);
      } else if (!(s.f[mm].g - 1.0 == 0.0 && s.f[mm].d == 0.0)) {
        Fac g = s.f[mm];
        g.g -= 1.0;
        C.f.push_back(std::move(g));
      }
    }
    C.f.push_back(std::move(D));
    const int rc = expand(C, out, depth + 1, err);
    if (rc != SDI_OK) return rc;
  }
  return SDI_OK;
}

}  // namespace

int expand_poles(const sdi_problem_desc* d, PoleExpansion& X, std::string& err) {
  X = PoleExpansion{};
  for (int s = 0; s < d->nsectors; ++s) {
    const sdi_sector_desc& sd = d->sectors[s];
    bool low = false;
    if (sd.mono_a)
      for (int j = 0; j < sd.nvars; ++j) low = low || sd.mono_a[j] < -1.0;
    if (!low) {
      X.descs.push_back(sd);
      std::vector<cplx> one(POLE_SERIES_LEN, 0.0);
      one[0] = 1.0;
      X.series.push_back(one);
      X.origin.push_back(s);
      continue;
    }
    const std::string where = "sector " + std::to_string(s) + ": ";
    if (d->complex_mode) {
      err = where + "a_j < -1 is reduced in real mode only";
      return SDI_ENOTSUP;
    }
    if (sd.term_coef_im) {
      err = where + "complex term coefficients need complex mode";
      return SDI_EINVAL;
    }
    const int n = sd.nvars;
    if (n < 1 || n > MAXV || sd.nfactors < 0 || sd.nfactors > MAXF || !sd.mono_b ||
        (sd.nfactors && (!sd.fac_nterms || !sd.fac_gamma || !sd.fac_delta || !sd.term_coef || !sd.term_exps))) {
      err = where + "malformed sector";
      return SDI_EINVAL;
    }
    Sec S0{n, std::vector<double>(sd.mono_a, sd.mono_a + n), std::vector<double>(sd.mono_b, sd.mono_b + n), {}, {},
           sd.coeff_re, sd.coeff_im};
    S0.series.assign(POLE_SERIES_LEN, 0.0);
    S0.series[0] = 1.0;
    size_t t0 = 0;
    for (int m = 0; m < sd.nfactors; ++m) {
      const int T = sd.fac_nterms[m];
      if (T < 1) {
        err = where + "empty factor";
        return SDI_EINVAL;
      }
      const double g = sd.fac_gamma[m], dl = sd.fac_delta[m];
      // derivative factors can vanish where the evaluator takes logarithms
      // unless every exponent is an integer (integer powers by products)
      if (g != std::floor(g) || dl != std::floor(dl)) {
        err = where + "a_j < -1 is reduced only for integer factor exponents";
        return SDI_ENOTSUP;
      }
      Fac f{g, dl, std::vector<double>(sd.term_coef + t0, sd.term_coef + t0 + T),
            std::vector<uint8_t>(sd.term_exps + t0 * n, sd.term_exps + (t0 + T) * n)};
      S0.f.push_back(std::move(f));
      t0 += T;
    }
    std::vector<Sec> parts;
    const int rc = expand(S0, parts, 0, err);
    if (rc != SDI_OK) {
      err = where + err;
      return rc;
    }
    for (Sec& p : parts) {
      if ((int)p.f.size() > MAXF) {
        err = where + "reducing a_j < -1 needs more than 4 factors";
        return SDI_ENOTSUP;
      }
      auto st = std::make_shared<PoleStore>();
      st->a = p.a;
      st->b = p.b;
      for (const Fac& f : p.f) {
        st->nterms.push_back((int32_t)f.coef.size());
        st->gam.push_back(f.g);
        st->del.push_back(f.d);
        st->coef.insert(st->coef.end(), f.coef.begin(), f.coef.end());
        st->exps.insert(st->exps.end(), f.exps.begin(), f.exps.end());
      }
      sdi_sector_desc o{};
      o.nvars = n;
      o.nfactors = (int32_t)p.f.size();
      o.deform_factor = -1;
      o.coeff_re = p.cre;
      o.coeff_im = p.cim;
      o.mono_a = st->a.data();
      o.mono_b = st->b.data();
      o.fac_nterms = st->nterms.data();
      o.fac_gamma = st->gam.data();
      o.fac_delta = st->del.data();
      o.term_coef = st->coef.data();
      o.term_exps = st->exps.data();
      X.store.push_back(st);
      X.descs.push_back(o);
      X.series.push_back(p.series);
      X.origin.push_back(s);
    }
  }
  return SDI_OK;
}

// SeparateTerms (section 4.4): the integrator receives the integrable terms of
// a sector one by one instead of its whole expression.  With the subtraction
// at x_j = 0 for the singular set S (a_j = -1), a sector is the sum over
// T subset S of
//   prod_{j in T} 1/(b_j eps) int prod_{j not in T} x_j^(a_j + b_j eps)
//       G(x with x_T = 0) dx,   the subtraction in S \ T keeping only the
//                               subtracted integrand,
// an integral over the n - |T| variables outside T: the factors keep the
// terms free of x_T (with the remaining exponent columns), the coefficient
// series takes prod 1/b_j, and shift = |T| records the eps^-|T|.  Parts come
// in the order of T as a bit mask over S in increasing variable index; a part
// left with no variable gets one constant variable (a = b = 0).  Sectors that
// fail the basic shape checks pass through unchanged (sdi_problem_create then
// reports them); a factor with no term on a face is refused (SDI_ENOTSUP).
int separate_terms(PoleExpansion& X, std::string& err) {
  PoleExpansion Y;
  for (size_t p = 0; p < X.descs.size(); ++p) {
    const sdi_sector_desc& sd = X.descs[p];
    const int n = sd.nvars;
    bool ok = n >= 1 && n <= MAXV && sd.nfactors >= 0 && sd.nfactors <= MAXF && sd.mono_a && sd.mono_b &&
              (!sd.nfactors || (sd.fac_nterms && sd.fac_gamma && sd.fac_delta));
    std::vector<int> S;
    size_t nt_all = 0;
    if (ok) {
      for (int m = 0; m < sd.nfactors; ++m) {
        ok = ok && sd.fac_nterms[m] >= 0;
        if (ok) nt_all += (size_t)sd.fac_nterms[m];
      }
      ok = ok && (nt_all == 0 || (sd.term_coef && sd.term_exps));
      for (int j = 0; ok && j < n; ++j)
        if (sd.mono_a[j] == -1.0) {
          S.push_back(j);
          ok = std::isfinite(sd.mono_b[j]) && sd.mono_b[j] != 0.0;
        }
      ok = ok && (int)S.size() <= MAXS;
    }
    if (!ok || S.empty()) {
      Y.descs.push_back(sd);
      Y.series.push_back(X.series[p]);
      Y.origin.push_back(X.origin[p]);
      Y.shift.push_back(0);
      Y.sub_only.push_back(0);
      continue;
    }
    const int ns = (int)S.size();
    for (int T = 0; T < (1 << ns); ++T) {
      std::vector<char> inT(n, 0);
      double scale = 1.0;
      for (int i = 0; i < ns; ++i)
        if (T >> i & 1) {
          inT[S[i]] = 1;
          scale /= sd.mono_b[S[i]];
        }
      std::vector<int> keep;
      for (int j = 0; j < n; ++j)
        if (!inT[j]) keep.push_back(j);
      const bool dummy = keep.empty();
      const int nf = dummy ? 1 : (int)keep.size();
      auto st = std::make_shared<PoleStore>();
      for (int j : keep) {
        st->a.push_back(sd.mono_a[j]);
        st->b.push_back(sd.mono_b[j]);
        st->dmono.push_back(sd.deform_mono ? sd.deform_mono[j] : 0);
      }
      if (dummy) {
        st->a.push_back(0.0);
        st->b.push_back(0.0);
        st->dmono.push_back(0);
      }
      size_t t0 = 0;
      for (int m = 0; m < sd.nfactors; ++m) {
        int kept = 0;
        for (int t = 0; t < sd.fac_nterms[m]; ++t) {
          const uint8_t* e = sd.term_exps + (t0 + t) * (size_t)n;
          bool on_face = true;
          for (int j = 0; j < n; ++j) on_face = on_face && !(inT[j] && e[j] != 0);
          if (!on_face) continue;
          st->coef.push_back(sd.term_coef[t0 + t]);
          for (int j : keep) st->exps.push_back(e[j]);
          if (dummy) st->exps.push_back(0);
          ++kept;
        }
        if (kept == 0) {
          err = "sector " + std::to_string(X.origin[p]) + ": factor " + std::to_string(m) +
                " has no term on the face x_j = 0 of a separated term";
          return SDI_ENOTSUP;
        }
        st->nterms.push_back(kept);
        st->gam.push_back(sd.fac_gamma[m]);
        st->del.push_back(sd.fac_delta[m]);
        t0 += (size_t)sd.fac_nterms[m];
      }
      sdi_sector_desc o = sd;
      o.nvars = nf;
      o.mono_a = st->a.data();
      o.mono_b = st->b.data();
      o.deform_mono = sd.deform_mono ? st->dmono.data() : nullptr;
      o.fac_nterms = st->nterms.data();
      o.fac_gamma = st->gam.data();
      o.fac_delta = st->del.data();
      o.term_coef = st->coef.empty() ? nullptr : st->coef.data();
      o.term_exps = st->exps.empty() ? nullptr : st->exps.data();
      o.term_coef_im = nullptr;
      std::vector<cplx> ser = X.series[p];
      for (cplx& c : ser) c *= scale;
      Y.store.push_back(st);
      Y.descs.push_back(o);
      Y.series.push_back(ser);
      Y.origin.push_back(X.origin[p]);
      Y.shift.push_back(__builtin_popcount(T));
      Y.sub_only.push_back(1);
    }
  }
  for (auto& st : X.store) Y.store.push_back(st);
  X = std::move(Y);
  return SDI_OK;
}

}  // namespace sdi
