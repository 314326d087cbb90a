// Laurent series of the Feynman prefactor of eq. (2) with (i pi^(d/2))^l and
// exp(-l gamma_E eps) pulled out (section 4.3):
//   Pi(eps) = exp(l gamma_E eps) Gamma(A - l d0/2 + l eps) / prod_i Gamma(a_i).
// Series arithmetic in long double from
//   ln Gamma(1 + x) = -gamma_E x + sum_{k>=2} (-1)^k zeta(k) x^k / k,
//   Gamma(N + x) = Gamma(1 + x) prod_{k=1}^{N-1} (k + x)    (N >= 1),
//   Gamma(N + x) = Gamma(1 + x) / prod_{k=N}^{0} (k + x)     (N <= 0),
// with zeta(k) from the Euler-Maclaurin formula.
#include <cmath>
#include <vector>

#include "host.h"

namespace sdi {

typedef long double LD;

static LD zeta_em(int s) {
  const int N = 24;
  LD sum = 0;
  for (int n = 1; n < N; ++n) sum += powl((LD)n, -(LD)s);
  const LD Nl = N;
  sum += powl(Nl, 1 - (LD)s) / (s - 1) + powl(Nl, -(LD)s) / 2;
  // Bernoulli numbers B_2 .. B_16 over (2j)!
  static const LD B[] = {1.0L / 6, -1.0L / 30, 1.0L / 42, -1.0L / 30, 5.0L / 66, -691.0L / 2730, 7.0L / 6,
                         -3617.0L / 510};
  LD fact = 1;   // (2j)!
  LD rising = s; // s (s+1) ... (s+2j-2)
  for (int j = 1; j <= 8; ++j) {
    fact *= (LD)(2 * j - 1) * (2 * j);
    if (j > 1) rising *= (LD)(s + 2 * j - 3) * (s + 2 * j - 2);
    sum += B[j - 1] / fact * rising * powl(Nl, -(LD)s - 2 * j + 1);
  }
  return sum;
}

static std::vector<LD> mul(const std::vector<LD>& a, const std::vector<LD>& b, size_t n) {
  std::vector<LD> o(n, 0);
  for (size_t i = 0; i < a.size() && i < n; ++i)
    for (size_t j = 0; j < b.size() && i + j < n; ++j) o[i + j] += a[i] * b[j];
  return o;
}

static std::vector<LD> inv(const std::vector<LD>& a, size_t n) {
  std::vector<LD> o(n, 0);
  o[0] = 1 / a[0];
  for (size_t k = 1; k < n; ++k) {
    LD s = 0;
    for (size_t j = 1; j <= k && j < a.size(); ++j) s += a[j] * o[k - j];
    o[k] = -s / a[0];
  }
  return o;
}

static std::vector<LD> exp_series(const std::vector<LD>& c, size_t n) {
  // c[0] == 0; E' = c' E  =>  k E_k = sum_{j=1}^{k} j c_j E_{k-j}
  std::vector<LD> e(n, 0);
  e[0] = 1;
  for (size_t k = 1; k < n; ++k) {
    LD s = 0;
    for (size_t j = 1; j <= k && j < c.size(); ++j) s += (LD)j * c[j] * e[k - j];
    e[k] = s / (LD)k;
  }
  return e;
}

int prefactor_series(int loops, const int32_t* idx, int nprops, int d0, int len, int* lead, double* out,
                     std::string& err) {
  if (loops < 1 || nprops < 1 || len < 1 || len > 64 || !idx || !lead || !out) {
    err = "prefactor: need loops >= 1, nprops >= 1, 1 <= len <= 64 and non-null arrays";
    return SDI_EINVAL;
  }
  long A = 0;
  for (int i = 0; i < nprops; ++i) {
    if (idx[i] < 1) {
      err = "prefactor: indices must be >= 1";
      return SDI_EINVAL;
    }
    A += idx[i];
  }
  if ((loops * d0) % 2) {
    err = "prefactor: l*d0 must be even";
    return SDI_ENOTSUP;
  }
  const long N0 = A - (long)loops * d0 / 2;
  const size_t n = (size_t)len + 2;
  std::vector<LD> c(n, 0);
  for (size_t k = 2; k < n; ++k) c[k] = ((k % 2) ? -1 : 1) * zeta_em((int)k) * powl((LD)loops, (LD)k) / (LD)k;
  std::vector<LD> ser = exp_series(c, n);
  int ld = 0;
  if (N0 >= 1) {
    for (long k = 1; k < N0; ++k) ser = mul(ser, {(LD)k, (LD)loops}, n);
  } else {
    std::vector<LD> den = {1};
    for (long k = N0; k < 0; ++k) den = mul(den, {(LD)k, (LD)loops}, n);
    ser = mul(ser, inv(den, n), n);
    for (auto& v : ser) v /= loops;
    ld = -1;
  }
  LD norm = 1;
  for (int i = 0; i < nprops; ++i)
    for (int k = 2; k < idx[i]; ++k) norm *= k;
  for (int i = 0; i < len; ++i) out[i] = (double)(ser[i] / norm);
  *lead = ld;
  return SDI_OK;
}

}  // namespace sdi
