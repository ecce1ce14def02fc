// Host-side moments of the weight exp(-x^beta) and the rational form of beta.
// No device code: the library includes it through its internal header, and
// the CPU-only sanitizer build of the tests compiles it on its own.
#pragma once
#include <cstdint>
#include <vector>

#include "hk_mp.hpp"

namespace hk {

// beta = num/den in lowest terms as p/q; false unless num, den >= 1
bool reduce_beta(int64_t num, int64_t den, uint32_t* p, uint32_t* q);
// log2 of mu_n = (1/beta) Gamma((n+1)/beta) in double precision (sizes only)
double log2_mu(int n, uint32_t p, uint32_t q);
// X_n = RNE(2^K mu_n) for n = 0..2N-2, correctly rounded; false if the
// rounding of some moment stays undecided at the largest working precision
bool build_moments(int N, uint32_t p, uint32_t q, int K, std::vector<MP>& X);

}  // namespace hk
