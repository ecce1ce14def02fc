// Rigorous inertia of M - xI around the fixed-point factorisation (the
// paper's "Interval Verification", in midpoint-radius form).  The midpoints
// are the factors the GPU computed (C, L, pivots); a radius per entry bounds
// the distance to the same quantity of the exact elimination of the true
// matrix (true moments, x exact):
//   A^(0):   rho = 2^-(K+1) (correctly rounded moments);
//   column k: eC[r] = rho[r][k] + 2^-(h+1) (the rounding of C), eD = eC[k];
//            with d = the pivot and d > eD,
//            eL[r] = (eC[r] + |C[r]|/d eD) / (d - eD) + 2^-(h+1);
//   update:  rho[r][c] += |C[c]| eL[r] + eC[c] (|L[r]| + eL[r]).
// A pivot is certified positive when d > eD, negative when d < -eD.  The
// magnitudes |C| and |L| come from a kernel that bounds each entry from its
// top digits; the recursion runs on the host in (double, exponent) numbers
// with every operation rounded up (round to nearest, then one ulp up), so
// every radius bounds the exact recursion from above.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "hk_internal.hpp"

namespace hk {
namespace {

// x = m 2^e, m in [1, 2) or m = 0
struct Ex {
  double m = 0;
  int64_t e = 0;
};

inline Ex ex_norm(double m, int64_t e) {
  Ex r;
  if (m == 0) return r;
  int t = 0;
  r.m = std::frexp(m, &t) * 2.0;   // [1, 2)
  r.e = e + t - 1;
  return r;
}
inline double up(double x) { return std::nextafter(x, INFINITY); }
inline double down(double x) { return std::nextafter(x, 0.0); }
inline Ex ex_pow2(int64_t e) { Ex r; r.m = 1; r.e = e; return r; }
inline Ex mul_up(const Ex& a, const Ex& b) {
  if (a.m == 0 || b.m == 0) return Ex();
  return ex_norm(up(a.m * b.m), a.e + b.e);
}
inline Ex div_up(const Ex& a, const Ex& b) { return ex_norm(up(a.m / b.m), a.e - b.e); }
inline Ex add_up(const Ex& a, const Ex& b) {
  if (a.m == 0) return b;
  if (b.m == 0) return a;
  const Ex& x = a.e >= b.e ? a : b;
  const Ex& y = a.e >= b.e ? b : a;
  const int64_t d = y.e - x.e;   // <= 0
  const double t = d < -1100 ? 0.0 : std::ldexp(y.m, (int)d);
  return ex_norm(up(x.m + t), x.e);
}
// a - b rounded down, for a > b >= 0 (m = 0 when b >= a)
inline Ex sub_down(const Ex& a, const Ex& b) {
  if (b.m == 0) return a;
  if (b.e > a.e) return Ex();
  const int64_t d = b.e - a.e;
  const double t = d < -1100 ? 0.0 : std::ldexp(b.m, (int)d);
  const double r = down(a.m - t);
  return r > 0 ? ex_norm(r, a.e) : Ex();
}
inline int ex_cmp(const Ex& a, const Ex& b) {
  if (a.m == 0 || b.m == 0) return a.m == 0 ? (b.m == 0 ? 0 : -1) : 1;
  if (a.e != b.e) return a.e < b.e ? -1 : 1;
  return a.m < b.m ? -1 : (a.m > b.m ? 1 : 0);
}
inline double ex_log2(const Ex& a) { return a.m == 0 ? -INFINITY : std::log2(a.m) + (double)a.e; }

// bounds of |v| for an exact integer v (host MP): lo <= |v| <= hi
void mp_bounds(const MP& v, Ex& lo, Ex& hi) {
  lo = hi = Ex();
  if (v.d.empty()) return;
  const int64_t bl = v.bitlen();
  // the top 64 bits t, |v| in [t, t + 1) 2^(bl - 64)
  const int64_t sh = std::max<int64_t>(0, bl - 64);
  const MP t = shr_mag(v, sh);
  uint64_t w = 0;
  for (size_t i = 0; i < t.d.size() && i < 2; i++) w |= (uint64_t)t.d[i] << (32 * i);
  const double f = (double)w;   // rounded to nearest
  lo = ex_norm(down(f), sh);
  hi = ex_norm(up(up(f) + 1.0), sh);
}

struct Mag {
  double m;   // |value| <= m 2^e (units of the stored integer)
  int64_t e;
};

// upper bound of |sum_j d_j 2^(29 j)| over n balanced digits d[j * stride]:
// the top two digits exactly, the rest below 2^(29 (n - 2))
__device__ Mag top_bound(const int32_t* d, int n, int64_t stride) {
  Mag r;
  while (n > 0 && d[(int64_t)(n - 1) * stride] == 0) n--;
  if (n == 0) { r.m = 0; r.e = 0; return r; }
  if (n <= 2) {
    const int64_t v = (int64_t)d[(int64_t)(n - 1) * stride] * (n == 2 ? (int64_t)1 << DB : 1) +
                      (n == 2 ? (int64_t)d[0] : 0);
    r.m = fabs((double)v);
    r.e = 0;
    return r;
  }
  const int64_t hi = (int64_t)d[(int64_t)(n - 1) * stride] * ((int64_t)1 << DB) + d[(int64_t)(n - 2) * stride];
  const double a = fabs((double)hi);   // |hi| < 2^58: one rounding
  r.m = nextafter(nextafter(a, INFINITY) + 1.0, INFINITY);
  r.e = (int64_t)DB * (n - 2);
  return r;
}

// one thread per factor entry (k, r >= k): bounds of |C_k[r]| and, for
// r > k, of |L_k[r]|, in units of 2^-h
__global__ void __launch_bounds__(256) k_magnitudes(const InstDesc* __restrict__ desc, Mag* magC, Mag* magL) {
  const InstDesc I = desc[0];
  const int k = blockIdx.y;
  const int N = I.N;
  const ColInfo kk = I.cols[k];
  for (int r = k + blockIdx.x * blockDim.x + threadIdx.x; r < N; r += gridDim.x * blockDim.x) {
    const int64_t ti = tri_index(N, k, r);
    const int nc = min(I.nC[ti], kk.CW);
    magC[ti] = top_bound(I.C + kk.coff + (int64_t)(r - k) * kk.CW, nc, 1);
    if (r > k) {
      const int nl = min(I.nL[ti], kk.LW);
      magL[ti] = top_bound(I.L + kk.loff + (r - k), nl, kk.R);
    } else {
      magL[ti].m = 0;
      magL[ti].e = 0;
    }
  }
}

}  // namespace

hk_status certify_factor(hk_matrix m, hipStream_t s, const std::vector<MP>& piv, int* n_negative,
                         int* certified, double* min_margin, double* margins) {
  const Plan& P = m->P;
  const int N = P.N, h = P.h, K = P.K;
  // the magnitudes, in the working triangle (free once the factors are out)
  const size_t need = 2 * sizeof(Mag) * (size_t)P.ntri;
  if (P.o_K - P.o_A < need) { g_err = "certify: working triangle too small"; return HK_EINVAL; }
  Mag* dC = (Mag*)m->D.A;
  Mag* dL = dC + P.ntri;
  hipLaunchKernelGGL(k_magnitudes, dim3((N + 255) / 256, N), dim3(256), 0, s, m->D.desc, dC, dL);
  std::vector<Mag> hC(P.ntri), hL(P.ntri);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hC.data(), dC, sizeof(Mag) * P.ntri, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hL.data(), dL, sizeof(Mag) * P.ntri, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { g_err = std::string("certify: ") + hipGetErrorString(e); return HK_EDEVICE; }
  auto magC = [&](int k, int r) { const Mag& g = hC[tri_index(N, k, r)]; return ex_norm(g.m, g.e - h); };
  auto magL = [&](int k, int r) { const Mag& g = hL[tri_index(N, k, r)]; return ex_norm(g.m, g.e - h); };
  const Ex half = ex_pow2(-(int64_t)h - 1);
  // rho, column by column: rho[c][r - c]
  std::vector<std::vector<Ex>> rho(N);
  for (int c = 0; c < N; c++) rho[c].assign(N - c, ex_pow2(-(int64_t)K - 1));
  int nneg = 0, ok = 1;
  double mmin = INFINITY;
  const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  std::vector<Ex> eC, eL, Cc, Sl;
  for (int k = 0; k < N; k++) {
    eC.assign(N - k, Ex());
    for (int r = k; r < N; r++) eC[r - k] = add_up(rho[k][r - k], half);
    Ex dlo, dhi;
    mp_bounds(piv[k], dlo, dhi);
    dlo = ex_norm(dlo.m, dlo.e - h);
    dhi = ex_norm(dhi.m, dhi.e - h);
    const Ex eD = eC[0];
    const bool neg = piv[k].neg && !piv[k].d.empty();
    const double margin = ex_log2(dlo) - ex_log2(eD);
    if (margins) margins[k] = margin;
    mmin = std::min(mmin, margin);
    if (ex_cmp(dlo, eD) <= 0) { ok = 0; }
    if (neg) nneg++;
    if (k == N - 1) break;
    if (neg || !ok) {
      // a pivot before the last column that is negative, or not certified:
      // the radii beyond it are not bounded (the margin so far stays, as a
      // lower estimate of what is missing; a negative pivot has none)
      ok = 0;
      for (int j = k + 1; j < N; j++) if (margins) margins[j] = -INFINITY;
      if (neg) mmin = -INFINITY;
      break;
    }
    // eL[r] = (eC[r] + |C[r]|/d eD) / (d - eD) + 2^-(h+1), with d from below
    const Ex den = sub_down(dlo, eD);
    eL.assign(N - k, Ex());
    Cc.assign(N - k, Ex());
    Sl.assign(N - k, Ex());
    for (int r = k + 1; r < N; r++) {
      const Ex Cr = magC(k, r);
      Cc[r - k] = Cr;
      const Ex num = add_up(eC[r - k], mul_up(div_up(Cr, dlo), eD));
      eL[r - k] = add_up(div_up(num, den), half);
      Sl[r - k] = add_up(magL(k, r), eL[r - k]);
    }
    // rho[c][r] += |C[c]| eL[r] + eC[c] (|L[r]| + eL[r]), c in (k, N), r >= c
    auto work = [&](int t) {
      for (int c = k + 1 + t; c < N; c += nth) {
        const Ex cc = Cc[c - k], ec = eC[c - k];
        std::vector<Ex>& col = rho[c];
        for (int r = c; r < N; r++)
          col[r - c] = add_up(col[r - c], add_up(mul_up(cc, eL[r - k]), mul_up(ec, Sl[r - k])));
      }
    };
    if ((int64_t)(N - k) * (N - k) < 20000 || nth == 1) {
      for (int t = 0; t < nth; t++) work(t);
    } else {
      std::vector<std::thread> th;
      for (int t = 0; t < nth; t++) th.emplace_back(work, t);
      for (auto& x : th) x.join();
    }
  }
  // the last pivot: certified when |d| > eD whatever its sign
  if (n_negative) *n_negative = nneg;
  if (certified) *certified = ok;
  if (min_margin) *min_margin = mmin;
  return HK_OK;
}

}  // namespace hk

using namespace hk;

extern "C" hk_status hk_certify(hk_matrix m, hipStream_t s, int* n_negative, int* certified, double* min_margin_bits,
                                double* margin_bits) {
  if (!m) { g_err = "null matrix"; return HK_EINVAL; }
  if (!m->factored) { g_err = "no factorisation"; return HK_EINVAL; }
  const int N = m->P.N;
  const int64_t nd = hk_factor_export(m, 2, 0, N, nullptr, nullptr, nullptr, 0, s);
  if (nd < 0) return HK_EDEVICE;
  std::vector<int32_t> slen(N);
  std::vector<int64_t> off(N);
  std::vector<uint32_t> dig(std::max<int64_t>(nd, 1));
  if (hk_factor_export(m, 2, 0, N, slen.data(), off.data(), dig.data(), (int64_t)dig.size(), s) < 0) return HK_EDEVICE;
  std::vector<MP> piv(N);
  for (int k = 0; k < N; k++) {
    const int n = slen[k] < 0 ? -slen[k] : slen[k];
    piv[k].d.assign(dig.begin() + off[k], dig.begin() + off[k] + n);
    piv[k].trim();
    piv[k].neg = slen[k] < 0 && !piv[k].d.empty();
  }
  double mm = 0;
  int nn = 0, ok = 0;
  const hk_status st = certify_factor(m, s, piv, &nn, &ok, &mm, margin_bits);
  if (st != HK_OK) return st;
  if (n_negative) *n_negative = nn;
  if (certified) *certified = ok;
  if (min_margin_bits) *min_margin_bits = mm;
  return HK_OK;
}
