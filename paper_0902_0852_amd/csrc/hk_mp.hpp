// Host-side multiprecision integers of the hk library (sign + magnitude,
// base-2^32 digits).  Used only for setup and driver arithmetic: the moment
// constants, the eigenvalue iterates and decimal formatting.  Every O(N^3)
// and O(N^2) step of the method runs in the HIP kernels.
#pragma once
#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

namespace hk {

struct MP {
  bool neg = false;
  std::vector<uint32_t> d;  // little endian, no leading zeros

  MP() = default;
  static MP from_u64(uint64_t v) {
    MP r;
    while (v) { r.d.push_back((uint32_t)v); v >>= 32; }
    return r;
  }
  static MP from_i64(int64_t v) {
    MP r = from_u64(v < 0 ? (uint64_t)(-(v + 1)) + 1 : (uint64_t)v);
    r.neg = v < 0 && !r.d.empty();
    return r;
  }
  bool is_zero() const { return d.empty(); }
  int sign() const { return d.empty() ? 0 : (neg ? -1 : 1); }
  void trim() {
    while (!d.empty() && d.back() == 0) d.pop_back();
    if (d.empty()) neg = false;
  }
  int64_t bitlen() const {
    if (d.empty()) return 0;
    return 32 * (int64_t)(d.size() - 1) + (32 - __builtin_clz(d.back()));
  }
  bool bit(int64_t i) const {
    size_t w = (size_t)(i >> 5);
    return w < d.size() && ((d[w] >> (i & 31)) & 1u);
  }
};

// |a| vs |b|
inline int cmp_mag(const MP& a, const MP& b) {
  if (a.d.size() != b.d.size()) return a.d.size() < b.d.size() ? -1 : 1;
  for (size_t i = a.d.size(); i-- > 0;)
    if (a.d[i] != b.d[i]) return a.d[i] < b.d[i] ? -1 : 1;
  return 0;
}
inline int cmp(const MP& a, const MP& b) {
  int sa = a.sign(), sb = b.sign();
  if (sa != sb) return sa < sb ? -1 : 1;
  int m = cmp_mag(a, b);
  return sa >= 0 ? m : -m;
}

inline MP add_mag(const MP& a, const MP& b) {
  const MP& x = a.d.size() >= b.d.size() ? a : b;
  const MP& y = a.d.size() >= b.d.size() ? b : a;
  MP r;
  r.d.resize(x.d.size() + 1);
  uint64_t c = 0;
  for (size_t i = 0; i < x.d.size(); i++) {
    c += (uint64_t)x.d[i] + (i < y.d.size() ? y.d[i] : 0u);
    r.d[i] = (uint32_t)c;
    c >>= 32;
  }
  r.d[x.d.size()] = (uint32_t)c;
  r.trim();
  return r;
}
// |a| - |b| assuming |a| >= |b|
inline MP sub_mag(const MP& a, const MP& b) {
  MP r;
  r.d.resize(a.d.size());
  int64_t br = 0;
  for (size_t i = 0; i < a.d.size(); i++) {
    int64_t t = (int64_t)a.d[i] - (i < b.d.size() ? (int64_t)b.d[i] : 0) - br;
    br = t < 0;
    r.d[i] = (uint32_t)(t & 0xffffffffLL);
  }
  r.trim();
  return r;
}
inline MP add(const MP& a, const MP& b) {
  if (a.neg == b.neg) { MP r = add_mag(a, b); r.neg = a.neg && !r.d.empty(); return r; }
  int c = cmp_mag(a, b);
  if (c == 0) return MP();
  MP r = c > 0 ? sub_mag(a, b) : sub_mag(b, a);
  r.neg = (c > 0 ? a.neg : b.neg) && !r.d.empty();
  return r;
}
inline MP neg(MP a) { if (!a.d.empty()) a.neg = !a.neg; return a; }
inline MP sub(const MP& a, const MP& b) { return add(a, neg(b)); }

// 32-bit digit vectors as 64-bit limbs and back (leading zeros dropped)
inline std::vector<uint64_t> limbs64(const std::vector<uint32_t>& d) {
  std::vector<uint64_t> w((d.size() + 1) / 2, 0);
  for (size_t i = 0; i < d.size(); i++) w[i >> 1] |= (uint64_t)d[i] << (32 * (i & 1));
  while (!w.empty() && w.back() == 0) w.pop_back();
  return w;
}
inline std::vector<uint32_t> digits32(const uint64_t* w, size_t n) {
  std::vector<uint32_t> d(2 * n);
  for (size_t i = 0; i < n; i++) { d[2 * i] = (uint32_t)w[i]; d[2 * i + 1] = (uint32_t)(w[i] >> 32); }
  while (!d.empty() && d.back() == 0) d.pop_back();
  return d;
}

// schoolbook product, 64-bit limbs with 128-bit partial products
inline MP mul(const MP& a, const MP& b) {
  if (a.d.empty() || b.d.empty()) return MP();
  typedef unsigned __int128 u128;
  const std::vector<uint64_t> A = limbs64(a.d), B = limbs64(b.d);
  std::vector<uint64_t> R(A.size() + B.size(), 0);
  for (size_t i = 0; i < A.size(); i++) {
    uint64_t c = 0;
    const uint64_t ai = A[i];
    for (size_t j = 0; j < B.size(); j++) {
      // at most (2^64 - 1)^2 + 2 (2^64 - 1) = 2^128 - 1
      const u128 t = (u128)ai * B[j] + R[i + j] + c;
      R[i + j] = (uint64_t)t;
      c = (uint64_t)(t >> 64);
    }
    R[i + B.size()] = c;
  }
  MP r;
  r.d = digits32(R.data(), R.size());
  r.neg = a.neg != b.neg && !r.d.empty();
  return r;
}
inline MP mul_small(const MP& a, uint32_t m) {
  MP r;
  if (a.d.empty() || m == 0) return r;
  r.d.resize(a.d.size() + 1);
  uint64_t c = 0;
  for (size_t i = 0; i < a.d.size(); i++) {
    uint64_t t = (uint64_t)a.d[i] * m + c;
    r.d[i] = (uint32_t)t;
    c = t >> 32;
  }
  r.d[a.d.size()] = (uint32_t)c;
  r.neg = a.neg;
  r.trim();
  return r;
}
// magnitude divided by a small divisor, remainder returned
inline MP divmod_small(const MP& a, uint32_t m, uint32_t* rem) {
  MP q;
  q.d.resize(a.d.size());
  uint64_t r = 0;
  for (size_t i = a.d.size(); i-- > 0;) {
    uint64_t cur = (r << 32) | a.d[i];
    q.d[i] = (uint32_t)(cur / m);
    r = cur % m;
  }
  q.neg = a.neg;
  q.trim();
  if (rem) *rem = (uint32_t)r;
  return q;
}
inline MP shl(const MP& a, int64_t s) {
  if (a.d.empty() || s == 0) return a;
  size_t w = (size_t)(s >> 5);
  int b = (int)(s & 31);
  MP r;
  r.d.assign(a.d.size() + w + 1, 0u);
  for (size_t i = 0; i < a.d.size(); i++) {
    uint64_t v = (uint64_t)a.d[i] << b;
    r.d[i + w] |= (uint32_t)v;
    r.d[i + w + 1] |= (uint32_t)(v >> 32);
  }
  r.neg = a.neg;
  r.trim();
  return r;
}
// floor(|a| / 2^s) with the sign of a (truncation of the magnitude)
inline MP shr_mag(const MP& a, int64_t s) {
  size_t w = (size_t)(s >> 5);
  int b = (int)(s & 31);
  if (w >= a.d.size()) return MP();
  MP r;
  r.d.resize(a.d.size() - w);
  for (size_t i = 0; i < r.d.size(); i++) {
    uint64_t v = a.d[i + w];
    if (i + w + 1 < a.d.size()) v |= (uint64_t)a.d[i + w + 1] << 32;
    r.d[i] = (uint32_t)(v >> b);
  }
  r.neg = a.neg;
  r.trim();
  return r;
}
inline bool low_bits_zero(const MP& a, int64_t s) {
  for (int64_t i = 0; i < s; i += 32) {
    size_t w = (size_t)(i >> 5);
    if (w >= a.d.size()) return true;
    uint32_t m = (s - i >= 32) ? 0xffffffffu : ((1u << (s - i)) - 1u);
    if (a.d[w] & m) return false;
  }
  return true;
}
inline MP inc_mag(MP a) {
  bool n = a.neg;
  a.neg = false;
  a = add_mag(a, MP::from_u64(1));
  a.neg = n && !a.d.empty();
  return a;
}

// Long division of magnitudes: returns q = floor(|a|/|b|), r = |a| - q|b|.
// Knuth's Algorithm D (The Art of Computer Programming, vol. 2, 4.3.1) in
// base 2^64 with a normalised divisor: the trial digit comes from the top
// two remainder digits and is corrected with the third, then an add-back.
inline void divmod_mag(const MP& a, const MP& b, MP& q, MP& r) {
  typedef unsigned __int128 u128;
  q = MP(); r = MP();
  if (cmp_mag(a, b) < 0) { r = a; r.neg = false; return; }
  if (b.d.size() == 1) {
    uint32_t rr;
    MP aa = a; aa.neg = false;
    q = divmod_small(aa, b.d[0], &rr);
    r = MP::from_u64(rr);
    return;
  }
  const std::vector<uint64_t> A = limbs64(a.d), B = limbs64(b.d);
  const size_t n = B.size();
  if (n == 1) {
    std::vector<uint64_t> Q(A.size());
    uint64_t rem = 0;
    for (size_t i = A.size(); i-- > 0;) {
      const u128 cur = ((u128)rem << 64) | A[i];
      Q[i] = (uint64_t)(cur / B[0]);
      rem = (uint64_t)(cur % B[0]);
    }
    q.d = digits32(Q.data(), Q.size());
    r.d = digits32(&rem, 1);
    return;
  }
  const int sh = __builtin_clzll(B[n - 1]);
  std::vector<uint64_t> Bn(n), R(A.size() + 1);
  for (size_t i = 0; i < n; i++) Bn[i] = (B[i] << sh) | (sh && i ? B[i - 1] >> (64 - sh) : 0);
  R[A.size()] = sh ? A.back() >> (64 - sh) : 0;
  for (size_t i = 0; i < A.size(); i++) R[i] = (A[i] << sh) | (sh && i ? A[i - 1] >> (64 - sh) : 0);
  const size_t m = R.size() - n;  // quotient digits
  std::vector<uint64_t> Q(m, 0);
  const uint64_t top = Bn[n - 1], nxt = Bn[n - 2];
  for (size_t j = m; j-- > 0;) {
    const u128 num = ((u128)R[j + n] << 64) | R[j + n - 1];
    u128 qh = num / top, rh = num % top;
    while ((qh >> 64) != 0 || qh * nxt > ((rh << 64) | R[j + n - 2])) {
      qh--; rh += top;
      if ((rh >> 64) != 0) break;
    }
    // R[j .. j+n] -= qd * Bn
    uint64_t qd = (uint64_t)qh, carry = 0, borrow = 0;
    for (size_t i = 0; i < n; i++) {
      const u128 p = (u128)qd * Bn[i] + carry;
      carry = (uint64_t)(p >> 64);
      const uint64_t pl = (uint64_t)p, x = R[j + i];
      const uint64_t t = x - pl;
      const uint64_t t2 = t - borrow;
      borrow = (uint64_t)(x < pl) + (uint64_t)(t < borrow);
      R[j + i] = t2;
    }
    const uint64_t x = R[j + n];
    const bool below = x < carry || x - carry < borrow;
    R[j + n] = x - carry - borrow;
    if (below) {
      qd--;
      uint64_t c = 0;
      for (size_t i = 0; i < n; i++) {
        const u128 s2 = (u128)R[j + i] + Bn[i] + c;
        R[j + i] = (uint64_t)s2;
        c = (uint64_t)(s2 >> 64);
      }
      R[j + n] += c;
    }
    Q[j] = qd;
  }
  q.d = digits32(Q.data(), Q.size());
  for (size_t i = 0; i < n; i++) R[i] = (R[i] >> sh) | (sh && i + 1 < n ? R[i + 1] << (64 - sh) : 0);
  r.d = digits32(R.data(), n);
}
inline MP floor_div(const MP& a, const MP& b) {  // floor(a/b), b > 0
  MP q, r;
  divmod_mag(a, b, q, r);
  if (a.neg) {
    if (!r.is_zero()) q = inc_mag(q);
    q.neg = !q.d.empty();
  }
  return q;
}
inline MP ceil_div(const MP& a, const MP& b) {  // ceil(a/b), b > 0
  return neg(floor_div(neg(a), b));
}
// round(a/b) to nearest, ties to even; b != 0
inline MP rne_div(const MP& a, const MP& b) {
  MP q, r;
  divmod_mag(a, b, q, r);
  MP r2 = shl(r, 1);
  int c = cmp_mag(r2, b);
  bool odd = !q.d.empty() && (q.d[0] & 1);
  if (c > 0 || (c == 0 && odd)) q = inc_mag(q);
  q.neg = (a.neg != b.neg) && !q.d.empty();
  return q;
}
inline MP rne_shr(const MP& a, int64_t s) {
  if (s <= 0) return shl(a, -s);
  MP q = shr_mag(a, s);
  bool half = a.bit(s - 1);
  bool sticky = !low_bits_zero(a, s - 1);
  bool odd = !q.d.empty() && (q.d[0] & 1);
  if (half && (sticky || odd)) { q = inc_mag(q); q.neg = a.neg && !q.d.empty(); }
  return q;
}
inline MP pow_small(uint32_t b, uint32_t e) {
  MP r = MP::from_u64(1);
  for (uint32_t i = 0; i < e; i++) r = mul_small(r, b);
  return r;
}

// decimal string of an integer
inline std::string to_dec(const MP& a) {
  if (a.d.empty()) return "0";
  MP t = a; t.neg = false;
  std::vector<uint32_t> chunks;
  while (!t.d.empty()) {
    uint32_t rr;
    t = divmod_small(t, 1000000000u, &rr);
    chunks.push_back(rr);
  }
  std::string s = a.neg ? "-" : "";
  s += std::to_string(chunks.back());
  for (size_t i = chunks.size() - 1; i-- > 0;) {
    std::string c = std::to_string(chunks[i]);
    s += std::string(9 - c.size(), '0') + c;
  }
  return s;
}
inline MP pow10(uint32_t e) { return pow_small(10, e); }

}  // namespace hk
