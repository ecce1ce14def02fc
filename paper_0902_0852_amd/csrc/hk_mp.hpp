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

inline MP mul(const MP& a, const MP& b) {
  if (a.d.empty() || b.d.empty()) return MP();
  MP r;
  r.d.assign(a.d.size() + b.d.size(), 0u);
  for (size_t i = 0; i < a.d.size(); i++) {
    uint64_t c = 0;
    const uint64_t ai = a.d[i];
    for (size_t j = 0; j < b.d.size(); j++) {
      uint64_t t = ai * b.d[j] + r.d[i + j] + c;
      r.d[i + j] = (uint32_t)t;
      c = t >> 32;
    }
    r.d[i + b.d.size()] = (uint32_t)c;
  }
  r.neg = a.neg != b.neg;
  r.trim();
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
// base 2^32 with a normalised divisor: the trial digit comes from the top
// two remainder digits and is corrected with the third, then an add-back.
inline void divmod_mag(const MP& a, const MP& b, MP& q, MP& r) {
  q = MP(); r = MP();
  if (cmp_mag(a, b) < 0) { r = a; r.neg = false; return; }
  if (b.d.size() == 1) {
    uint32_t rr;
    MP aa = a; aa.neg = false;
    q = divmod_small(aa, b.d[0], &rr);
    r = MP::from_u64(rr);
    return;
  }
  int sh = __builtin_clz(b.d.back());
  MP bn = shl(b, sh); bn.neg = false;
  MP an = shl(a, sh); an.neg = false;
  size_t n = bn.d.size();
  std::vector<uint32_t> rem(an.d.begin(), an.d.end());
  rem.push_back(0);
  size_t m = rem.size() - n;  // quotient digits
  q.d.assign(m, 0u);
  const uint64_t top = bn.d[n - 1], nxt = bn.d[n - 2];
  for (size_t jj = m; jj-- > 0;) {
    uint64_t hi2 = ((uint64_t)rem[jj + n] << 32) | rem[jj + n - 1];
    uint64_t qh = hi2 / top, rh = hi2 % top;
    while (qh > 0xffffffffULL || qh * nxt > ((rh << 32) | rem[jj + n - 2])) {
      qh--; rh += top;
      if (rh > 0xffffffffULL) break;
    }
    // rem[jj .. jj+n] -= qh * bn
    uint64_t carry = 0;
    int64_t borrow = 0;
    for (size_t i = 0; i < n; i++) {
      uint64_t p = qh * bn.d[i] + carry;
      carry = p >> 32;
      int64_t t = (int64_t)rem[jj + i] - (int64_t)(uint32_t)p - borrow;
      borrow = t < 0;
      rem[jj + i] = (uint32_t)(t & 0xffffffffLL);
    }
    int64_t t = (int64_t)rem[jj + n] - (int64_t)carry - borrow;
    rem[jj + n] = (uint32_t)(t & 0xffffffffLL);
    if (t < 0) {
      qh--;
      uint64_t c = 0;
      for (size_t i = 0; i < n; i++) {
        uint64_t s2 = (uint64_t)rem[jj + i] + bn.d[i] + c;
        rem[jj + i] = (uint32_t)s2;
        c = s2 >> 32;
      }
      rem[jj + n] += (uint32_t)c;
    }
    q.d[jj] = (uint32_t)qh;
  }
  q.trim();
  MP rr;
  rr.d.assign(rem.begin(), rem.begin() + n);
  rr.trim();
  r = shr_mag(rr, sh);
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
