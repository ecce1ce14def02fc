// CPU harness for the sanitizer build of the library's host arithmetic (test
// infrastructure): the correctly rounded moments and the multiprecision
// helpers the drivers use, compiled from the library's own sources under
// AddressSanitizer and UndefinedBehaviorSanitizer.  Results are printed in
// hexadecimal so that the test compares them with Python integers.
//
//   host_main moments N p q K   X_n, one per line
//   host_main mp SEED COUNT     for COUNT operand pairs (a, b) from a fixed
//                               xorshift sequence: a, b, |a| div |b|,
//                               |a| mod |b|, a*b, a+b, RNE(a/b), floor(a/b),
//                               ceil(a/b), RNE(a/2^s) with s, and a in decimal
#include "../../paper_0902_0852_amd/csrc/hk_moments.cpp"

#include <cstdio>
#include <cstdlib>

static std::string hex(const hk::MP& a) {
  if (a.d.empty()) return "0";
  char buf[16];
  std::string s = a.neg ? "-" : "";
  snprintf(buf, sizeof buf, "%x", a.d.back());
  s += buf;
  for (size_t i = a.d.size() - 1; i-- > 0;) {
    snprintf(buf, sizeof buf, "%08x", a.d[i]);
    s += buf;
  }
  return s;
}

static uint64_t st = 0x9e3779b97f4a7c15ull;
static uint64_t next() {
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return st;
}

// operands that reach the division's corner cases: top words near 2^32 or
// small, runs of all-ones and zero words, one-word divisors
static hk::MP operand(int maxw) {
  hk::MP r;
  const int n = 1 + (int)(next() % (uint64_t)maxw);
  const int shape = (int)(next() % 4);
  for (int i = 0; i < n; i++) {
    uint32_t w = (uint32_t)next();
    if (shape == 1) w = (next() % 3) ? 0xffffffffu : w;
    if (shape == 2) w = (next() % 3) ? 0u : w;
    r.d.push_back(w);
  }
  if (shape == 3) r.d.back() = 1 + (uint32_t)(next() % 7);
  r.neg = (next() & 1) != 0;
  r.trim();
  return r;
}

int main(int argc, char** argv) {
  if (argc == 6 && std::string(argv[1]) == "moments") {
    std::vector<hk::MP> X;
    if (!hk::build_moments(atoi(argv[2]), (uint32_t)atoi(argv[3]), (uint32_t)atoi(argv[4]), atoi(argv[5]), X))
      return 3;
    for (const hk::MP& x : X) printf("%s\n", hex(x).c_str());
    return 0;
  }
  if (argc == 4 && std::string(argv[1]) == "mp") {
    st ^= (uint64_t)atoll(argv[2]) * 0x2545f4914f6cdd1dull;
    const int count = atoi(argv[3]);
    for (int i = 0; i < count; i++) {
      const hk::MP a = operand(24), b0 = operand(12);
      const hk::MP b = b0.is_zero() ? hk::MP::from_u64(3) : b0;
      hk::MP bp = b;
      bp.neg = false;
      hk::MP q, r;
      hk::divmod_mag(a, b, q, r);
      const int64_t s = (int64_t)(next() % 700);
      printf("%s %s %s %s %s %s %s %s %s %lld %s %s\n", hex(a).c_str(), hex(b).c_str(), hex(q).c_str(),
             hex(r).c_str(), hex(hk::mul(a, b)).c_str(), hex(hk::add(a, b)).c_str(),
             hex(hk::rne_div(a, bp)).c_str(), hex(hk::floor_div(a, bp)).c_str(), hex(hk::ceil_div(a, bp)).c_str(),
             (long long)s, hex(hk::rne_shr(a, s)).c_str(), hk::to_dec(a).c_str());
    }
    return 0;
  }
  return 2;
}
