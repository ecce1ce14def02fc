// Correctly rounded fixed-point moments X_n = RNE(2^K mu_n) of the weight
// exp(-x^beta), mu_n = (1/beta) Gamma((n+1)/beta) (paper: the matrix
// definition in the Introduction, the moment form in "Properties of M").
//
// With beta = p/q in lowest terms and q(n+1) = m p + r (0 <= r < p):
//   r = 0:  mu_n = (q/p) (m-1)!                              (exact rational)
//   r > 0:  mu_n = (q/p) Gamma(r/p) prod_{j<m} (r + j p) / p^m
// so only Gamma(r/p), 0 < r < p, needs a transcendental evaluation.  It is
// taken from Gamma(s) = gamma(s, T) + Gamma(s, T), the lower part summed as
// the confluent series T^s e^{-T} sum_k T^k / (s)_{k+1} with T = u^p (so
// T^s = u^r is an integer), the upper part bounded by e^{-T}.  Each value
// comes with an explicit error bound; the rounded moment is accepted only if
// both ends of its error interval round to the same integer, otherwise the
// working precision grows (Ziv's strategy).
#include <cmath>
#include <vector>

#include "hk_internal.hpp"

namespace hk {

namespace {

// 2^F Gamma(r/p) ~ G with |2^F Gamma(r/p) - G| <= err
struct GammaApprox { MP G, err; };

GammaApprox gamma_rp(uint32_t r, uint32_t p, int64_t F) {
  double Tmin = (double)(F + 16) * std::log(2.0) + 4.0;
  uint32_t u = (uint32_t)std::ceil(std::pow(Tmin, 1.0 / p));
  if (u < 2) u = 2;
  while (std::pow((double)u, (double)p) < Tmin) u++;
  MP T = pow_small(u, p);
  // T fits in 32 bits for every realistic precision; larger T is refused by
  // the caller's precision cap.
  uint64_t Tv = 0;
  for (size_t i = T.d.size(); i-- > 0;) Tv = (Tv << 32) | T.d[i];
  const int64_t W = F + 96;
  // series S = 2^W sum_k T^k p^{k+1} / prod_{j<=k} (r + j p), floor chain
  MP t = divmod_small(shl(MP::from_u64(p), W), r, nullptr);
  MP t0 = t;
  MP S = t;
  uint64_t nS = 1;
  for (uint64_t k = 1;; k++) {
    uint64_t den = (uint64_t)r + k * (uint64_t)p;
    // multiply by T*p in two small steps to stay within 32-bit multipliers
    t = mul_small(mul_small(t, (uint32_t)Tv), p);
    if (den <= 0xffffffffULL) {
      t = divmod_small(t, (uint32_t)den, nullptr);
    } else {
      MP q, rr; divmod_mag(t, MP::from_u64(den), q, rr); t = q;
    }
    S = add(S, t);
    nS++;
    if (t.is_zero()) break;
  }
  // E = 2^W e^T, floor chain
  MP e = shl(MP::from_u64(1), W);
  MP E = e;
  uint64_t nE = 1;
  for (uint64_t k = 1;; k++) {
    e = mul_small(e, (uint32_t)Tv);
    if (k <= 0xffffffffULL) e = divmod_small(e, (uint32_t)k, nullptr);
    E = add(E, e);
    nE++;
    if (e.is_zero()) break;
  }
  // error bounds of the truncated floor chains (units of 2^-W):
  //   |dS| <= n^2 + n (S / t0 + 1),  |dE| <= n^2 + n (E / 2^W + 1)
  // plus the dropped tails, which are below one unit each once a term is 0
  MP nSq = MP::from_u64(nS), nEq = MP::from_u64(nE);
  MP errS = add(mul(nSq, nSq), mul(nSq, add(floor_div(S, t0), MP::from_u64(2))));
  MP errE = add(mul(nEq, nEq), mul(nEq, add(shr_mag(E, W), MP::from_u64(2))));
  MP ur = pow_small(u, r);
  MP num = shl(mul(ur, S), F);
  GammaApprox g;
  g.G = floor_div(num, E);
  // err <= u^r 2^F (errS E + S errE) / E^2 + 2^(F+W) / E + 2
  MP e1 = ceil_div(mul(shl(ur, F), add(mul(errS, E), mul(S, errE))), mul(E, E));
  MP e2 = ceil_div(shl(MP::from_u64(1), F + W), E);
  g.err = add(add(e1, e2), MP::from_u64(2));
  return g;
}

uint64_t gcd64(uint64_t a, uint64_t b) { while (b) { uint64_t t = a % b; a = b; b = t; } return a; }

}  // namespace

bool reduce_beta(int64_t num, int64_t den, uint32_t* p, uint32_t* q) {
  if (num < 1 || den < 1) return false;
  uint64_t g = gcd64((uint64_t)num, (uint64_t)den);
  uint64_t pp = (uint64_t)num / g, qq = (uint64_t)den / g;
  if (pp > 1000 || qq > 1000) return false;
  *p = (uint32_t)pp; *q = (uint32_t)qq;
  return true;
}

double log2_mu(int n, uint32_t p, uint32_t q) {
  double x = (double)q * (n + 1) / p;
  return (std::lgamma(x) + std::log((double)q / p)) / std::log(2.0);
}

bool build_moments(int N, uint32_t p, uint32_t q, int K, std::vector<MP>& X) {
  const int nmax = 2 * N - 2;
  double top = 0;
  for (int n = 0; n <= nmax; n++) top = std::max(top, log2_mu(n, p, q));
  int64_t guard = 64;
  for (int attempt = 0; attempt < 8; attempt++, guard *= 2) {
    const int64_t F = K + (int64_t)std::ceil(std::max(0.0, top)) + guard;
    std::vector<GammaApprox> gam(p);
    std::vector<bool> have(p, false);
    std::vector<MP> prod(p, MP::from_u64(1));
    std::vector<uint64_t> prod_m(p, 0);
    X.assign(nmax + 1, MP());
    bool ok = true;
    for (int n = 0; n <= nmax && ok; n++) {
      uint64_t a = (uint64_t)q * (uint64_t)(n + 1);
      uint64_t m = a / p, r = a % p;
      if (r == 0) {
        MP f = MP::from_u64(1);
        for (uint64_t i = 2; i < m; i++) f = mul_small(f, (uint32_t)i);
        X[n] = rne_div(shl(mul_small(f, q), K), MP::from_u64(p));
        continue;
      }
      if (!have[r]) { gam[r] = gamma_rp((uint32_t)r, p, F); have[r] = true; }
      while (prod_m[r] < m) { prod[r] = mul_small(prod[r], (uint32_t)(r + prod_m[r] * p)); prod_m[r]++; }
      MP den = shl(pow_small(p, (uint32_t)(m + 1)), F);
      MP base = shl(mul_small(prod[r], q), K);
      MP lo = rne_div(mul(base, sub(gam[r].G, gam[r].err)), den);
      MP hi = rne_div(mul(base, add(gam[r].G, gam[r].err)), den);
      if (cmp(lo, hi) != 0) { ok = false; break; }
      X[n] = lo;
    }
    if (ok) return true;
  }
  return false;
}

}  // namespace hk
