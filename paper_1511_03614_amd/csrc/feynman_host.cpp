// SDEvaluate[{U, F, l}, indices, order] (section 4.3): a Feynman integral
// given by its Symanzik polynomials, turned into sectors on the host and
// compiled like any other problem.
//
// Eq. (2): the integrand is prod_j x_j^(a_j - 1) U^(A - (l+1) d/2) /
// F^(A - l d/2) on the simplex, d = d0 - 2 eps, A = sum_j a_j; the prefactor
// exp(l gamma_E eps) Gamma(A - l d/2) / prod_j Gamma(a_j).  Primary sectors
// (section 4.2): x_k = 1 for each k, the other variables on the unit cube.
// Iterated decomposition (the classic strategy of the FIESTA papers, the S
// strategy of STRATEGY, section 4.4): while some polynomial, after its
// monomial factor is taken out, has no constant term, take the smallest set Z
// of variables (by size, then lexicographically) such that every term
// vanishes when they all do, and split into |Z| sectors: in sector k in Z,
// x_i -> x_i x_k for the other i in Z, which adds to the exponent of x_k the
// exponents of the others and the Jacobian x_k^(|Z| - 1).  Each final sector
// keeps the two polynomials with their monomials moved into the x_j powers;
// exponents a_j < -1 are reduced by sdi_problem_create.
#include <cmath>
#include <complex>
#include <map>

#include "host.h"
#include "kernels.h"

namespace sdi {

namespace {

using Exps = std::vector<int>;
using Coef = std::complex<double>;   // complex for complex masses (F's imaginary parts)

// A polynomial as its terms in insertion order (merging keeps the position of
// the first occurrence and adds coefficients in that order).
struct Poly {
  std::vector<std::pair<Exps, Coef>> terms;
  std::map<Exps, size_t> at;
  void add(const Exps& e, Coef c) {
    auto it = at.find(e);
    if (it == at.end()) {
      at.emplace(e, terms.size());
      terms.push_back({e, c});
    } else {
      terms[it->second].second += c;
    }
  }
  Poly nonzero() const {
    Poly o;
    for (auto& t : terms)
      if (t.second != Coef(0.0)) o.add(t.first, t.second);
    return o;
  }
};

Exps gcd_mono(const Poly& p) {
  Exps g = p.terms[0].first;
  for (auto& t : p.terms)
    for (size_t j = 0; j < g.size(); ++j) g[j] = std::min(g[j], t.first[j]);
  return g;
}

bool has_const(const Poly& p, const Exps& g) { return p.at.count(g) > 0; }

Poly substitute(const Poly& p, const std::vector<int>& Z, int k) {
  Poly o;
  for (auto& t : p.terms) {
    Exps e = t.first;
    for (int i : Z)
      if (i != k) e[k] += t.first[i];
    o.add(e, t.second);
  }
  return o.nonzero();
}

// Smallest Z (size, then lexicographic) hitting every term of p / x^g.
bool vanishing_set(const Poly& p, const Exps& g, std::vector<int>& Z) {
  const int n = (int)g.size();
  std::vector<Exps> red;
  for (auto& t : p.terms) {
    Exps e = t.first;
    for (int j = 0; j < n; ++j) e[j] -= g[j];
    red.push_back(e);
  }
  for (int size = 1; size <= n; ++size) {
    std::vector<int> idx(size);
    for (int i = 0; i < size; ++i) idx[i] = i;
    for (;;) {
      bool all = true;
      for (auto& e : red) {
        bool hit = false;
        for (int j : idx) hit = hit || e[j] > 0;
        if (!hit) {
          all = false;
          break;
        }
      }
      if (all) {
        Z = idx;
        return true;
      }
      int i = size - 1;
      while (i >= 0 && idx[i] == n - size + i) --i;
      if (i < 0) break;
      ++idx[i];
      for (int j = i + 1; j < size; ++j) idx[j] = idx[j - 1] + 1;
    }
  }
  return false;
}

struct State {
  std::vector<Poly> ps;
  std::vector<double> a, b;
  int depth;
};

struct OutSector {
  std::vector<double> a, b;
  std::vector<std::vector<Coef>> coef;
  std::vector<std::vector<uint8_t>> exps;   // [factor][term * n]
};

// The sectors of the integral: primary sectors in order k = 0..n-1, each
// decomposed depth first (the last split part first).
int decompose(const sdi_feynman_desc* d, std::vector<OutSector>& out, std::string& err) {
  const int n = d->nvars;
  int A = 0;
  for (int j = 0; j < n; ++j) A += d->indices[j];
  const double gU = A - (d->loops + 1) * d->d0 / 2.0, dU = d->loops + 1;
  const double gF = -(A - d->loops * d->d0 / 2.0), dF = -d->loops;
  const double gam[2] = {gU, gF}, del[2] = {dU, dF};
  Poly UF[2];
  for (int m = 0; m < 2; ++m) {
    const int nt = m == 0 ? d->u_nterms : d->f_nterms;
    const double* c = m == 0 ? d->u_coef : d->f_coef;
    const double* ci = m == 0 ? nullptr : d->f_coef_im;
    const uint8_t* e = m == 0 ? d->u_exps : d->f_exps;
    for (int t = 0; t < nt; ++t)
      UF[m].add(Exps(e + (size_t)t * n, e + (size_t)(t + 1) * n), Coef(c[t], ci ? ci[t] : 0.0));
    UF[m] = UF[m].nonzero();
  }
  for (int k = 0; k < n; ++k) {
    State st;
    for (int m = 0; m < 2; ++m) {
      Poly r;
      for (auto& t : UF[m].terms) {
        Exps e;
        for (int j = 0; j < n; ++j)
          if (j != k) e.push_back(t.first[j]);
        r.add(e, t.second);
      }
      st.ps.push_back(r.nonzero());
      if (st.ps.back().terms.empty()) {
        err = "U or F vanishes in primary sector " + std::to_string(k);
        return SDI_EINVAL;
      }
    }
    for (int j = 0; j < n; ++j)
      if (j != k) {
        st.a.push_back(d->indices[j] - 1.0);
        st.b.push_back(0.0);
      }
    st.depth = 0;
    std::vector<State> stack{st};
    while (!stack.empty()) {
      State s = stack.back();
      stack.pop_back();
      int bad = -1;
      for (int m = 0; m < 2 && bad < 0; ++m)
        if (!has_const(s.ps[m], gcd_mono(s.ps[m]))) bad = m;
      if (bad < 0) {
        OutSector o;
        o.a = s.a;
        o.b = s.b;
        const int nv = (int)s.a.size();
        for (int m = 0; m < 2; ++m) {
          const Exps g = gcd_mono(s.ps[m]);
          for (int j = 0; j < nv; ++j) {
            o.a[j] += g[j] * gam[m];
            o.b[j] += g[j] * del[m];
          }
          std::vector<std::pair<Exps, Coef>> terms = s.ps[m].terms;
          std::stable_sort(terms.begin(), terms.end(),
                           [](const std::pair<Exps, Coef>& x, const std::pair<Exps, Coef>& y) { return x.first < y.first; });
          std::vector<Coef> c;
          std::vector<uint8_t> e;
          for (auto& t : terms) {
            c.push_back(t.second);
            for (int j = 0; j < nv; ++j) {
              const int v = t.first[j] - g[j];
              if (v > 255) {
                err = "exponent above 255 after decomposition";
                return SDI_ENOTSUP;
              }
              e.push_back((uint8_t)v);
            }
          }
          o.coef.push_back(c);
          o.exps.push_back(e);
        }
        out.push_back(std::move(o));
        continue;
      }
      if (s.depth >= 40) {
        err = "sector decomposition did not terminate within 40 levels";
        return SDI_ENOTSUP;
      }
      std::vector<int> Z;
      if (!vanishing_set(s.ps[bad], gcd_mono(s.ps[bad]), Z)) {
        err = "a polynomial is identically zero";
        return SDI_EINVAL;
      }
      for (int k2 : Z) {
        State c;
        for (auto& q : s.ps) c.ps.push_back(substitute(q, Z, k2));
        c.a = s.a;
        c.b = s.b;
        for (int i : Z)
          if (i != k2) {
            c.a[k2] += s.a[i];
            c.b[k2] += s.b[i];
          }
        c.a[k2] += (double)Z.size() - 1.0;
        c.depth = s.depth + 1;
        for (auto& q : c.ps)
          if (q.terms.empty()) {
            err = "a polynomial vanished under decomposition";
            return SDI_EINVAL;
          }
        stack.push_back(std::move(c));
      }
    }
  }
  return SDI_OK;
}

int check_desc(const sdi_feynman_desc* d, std::string& err) {
  if (!d || !d->indices || !d->u_coef || !d->u_exps || !d->f_coef || !d->f_exps) {
    err = "feynman: null argument";
    return SDI_EINVAL;
  }
  if (d->nvars < 2 || d->nvars > MAXV + 1) {
    err = "feynman: nvars must be 2..17 (sectors have one variable fewer)";
    return SDI_EINVAL;
  }
  if (d->u_nterms < 1 || d->f_nterms < 1) {
    err = "feynman: U and F need terms";
    return SDI_EINVAL;
  }
  if (d->loops < 1 || d->loops > 8 || d->d0 < 1 || d->d0 > 12) {
    err = "feynman: loops must be 1..8 and d0 1..12";
    return SDI_EINVAL;
  }
  for (int j = 0; j < d->nvars; ++j)
    if (d->indices[j] < 1 || d->indices[j] > 8) {
      err = "feynman: indices must be 1..8";
      return SDI_EINVAL;
    }
  for (int t = 0; t < d->u_nterms + d->f_nterms; ++t) {
    const double c = t < d->u_nterms ? d->u_coef[t] : d->f_coef[t - d->u_nterms];
    const double ci = t >= d->u_nterms && d->f_coef_im ? d->f_coef_im[t - d->u_nterms] : 0.0;
    if (!std::isfinite(c) || !std::isfinite(ci)) {
      err = "feynman: coefficients must be finite";
      return SDI_EINVAL;
    }
  }
  if (d->f_coef_im && !d->complex_mode) {
    err = "feynman: complex F coefficients need complex mode";
    return SDI_EINVAL;
  }
  return SDI_OK;
}

int lowest_order(const std::vector<OutSector>& secs, const sdi_feynman_desc* d, int* pref_lead, std::string& err) {
  int lead = 0;
  double one = 0.0;
  const int rc = prefactor_series(d->loops, d->indices, d->nvars, d->d0, 1, &lead, &one, err);
  if (rc != SDI_OK) return rc;
  // singular variables after the reduction of a_j < -1: integer a_j <= -1 end at -1
  int ns = 0;
  for (auto& s : secs) {
    int c = 0;
    for (double v : s.a) c += v <= -1.0 && v == std::floor(v);
    ns = std::max(ns, c);
  }
  *pref_lead = lead;
  return lead - ns;
}

}  // namespace

}  // namespace sdi

using namespace sdi;

extern "C" {

int sdi_feynman_sectors(const sdi_feynman_desc* d, int32_t* nsectors, int32_t* order_min, int32_t* max_vars) {
  std::string err;
  int rc = check_desc(d, err);
  if (rc != SDI_OK) return rc;
  std::vector<OutSector> secs;
  rc = decompose(d, secs, err);
  if (rc != SDI_OK) return rc;
  int lead = 0;
  const int om = lowest_order(secs, d, &lead, err);
  if (!err.empty()) return SDI_EINVAL;
  if (nsectors) *nsectors = (int32_t)secs.size();
  if (order_min) *order_min = om;
  if (max_vars) *max_vars = d->nvars - 1;
  return SDI_OK;
}

int sdi_problem_from_feynman(sdi_ctx* ctx, const sdi_feynman_desc* d, sdi_problem** out) {
  if (!ctx || !out) return fail(ctx, SDI_EINVAL, "problem_from_feynman: null argument");
  *out = nullptr;
  std::string err;
  int rc = check_desc(d, err);
  if (rc != SDI_OK) return fail(ctx, rc, err);
  std::vector<OutSector> secs;
  rc = decompose(d, secs, err);
  if (rc != SDI_OK) return fail(ctx, rc, err);
  int lead = 0;
  const int om = lowest_order(secs, d, &lead, err);
  if (!err.empty()) return fail(ctx, SDI_EINVAL, err);
  if (d->order < om || d->order - om + 1 > KMAX)
    return fail(ctx, SDI_EINVAL, "order must lie in " + std::to_string(om) + ".." + std::to_string(om + KMAX - 1) +
                                     " (at most 8 orders from the leading pole)");
  int ns = lead - om;
  const int len = std::max(1, d->order - lead + ns + 1);
  std::vector<double> pref(len, 0.0), pim(len, 0.0);
  int lead2 = 0;
  rc = prefactor_series(d->loops, d->indices, d->nvars, d->d0, len, &lead2, pref.data(), err);
  if (rc != SDI_OK) return fail(ctx, rc, err);
  const int nv = d->nvars - 1;
  std::vector<sdi_sector_desc> sd(secs.size());
  std::vector<std::vector<int32_t>> nterms(secs.size());
  std::vector<std::vector<double>> coef(secs.size()), coef_im(secs.size()), gam(secs.size()), del(secs.size());
  std::vector<std::vector<uint8_t>> exps(secs.size());
  int A = 0;
  for (int j = 0; j < d->nvars; ++j) A += d->indices[j];
  const double gU = A - (d->loops + 1) * d->d0 / 2.0, dU = d->loops + 1;
  const double gF = -(A - d->loops * d->d0 / 2.0), dF = -d->loops;
  for (size_t s = 0; s < secs.size(); ++s) {
    for (int m = 0; m < 2; ++m) {
      nterms[s].push_back((int32_t)secs[s].coef[m].size());
      for (const Coef& c : secs[s].coef[m]) {
        coef[s].push_back(c.real());
        coef_im[s].push_back(c.imag());
      }
      exps[s].insert(exps[s].end(), secs[s].exps[m].begin(), secs[s].exps[m].end());
    }
    gam[s] = {gU, gF};
    del[s] = {dU, dF};
    sdi_sector_desc& x = sd[s];
    x = sdi_sector_desc{};
    x.nvars = nv;
    x.nfactors = 2;
    x.deform_factor = 1;
    x.coeff_re = 1.0;
    x.mono_a = secs[s].a.data();
    x.mono_b = secs[s].b.data();
    x.fac_nterms = nterms[s].data();
    x.fac_gamma = gam[s].data();
    x.fac_delta = del[s].data();
    x.term_coef = coef[s].data();
    x.term_exps = exps[s].data();
    x.term_coef_im = d->f_coef_im ? coef_im[s].data() : nullptr;
  }
  sdi_problem_desc pd{};
  pd.nsectors = (int32_t)secs.size();
  pd.sectors = sd.data();
  pd.order_min = om;
  pd.order_max = d->order;
  pd.pref_lead = lead2;
  pd.pref_len = len;
  pd.pref_re = pref.data();
  pd.pref_im = pim.data();
  pd.complex_mode = d->complex_mode;
  pd.lambda = d->lambda;
  return sdi_problem_create(ctx, &pd, out);
}

}  // extern "C"
