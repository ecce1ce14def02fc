// HIP kernels (gfx950) of the fixed-point LDL^T of M - xI.
//
// Number format on the device: balanced radix-2^29 digits in int32, value =
// sum_i d_i 2^(29 i).  Products of two digits are formed by v_mad_i64_i32
// (full rate on gfx950) and summed in int64 without carry handling: with
// |d| <= 2^28 every product is <= 2^56 in magnitude, so up to 96 products
// (plus a renormalised remainder) fit an int64 accumulator; accumulators are
// renormalised (split at bit 29, excess moved one column up) every 96
// products.  Negative numbers need no separate sign handling.
//
// Working triangle: column c holds rows r = c..N-1 as W_c digit planes of R_c
// (= N-c rounded up to 64) int32, so a wavefront of 64 consecutive rows reads
// one digit of 64 entries as one coalesced 256-byte line.  A trailing-update
// work item is (column c, 64-row tile t, output block q of WB = 16 digits);
// each item normalises its 16 digits and hands its carry to block q+1
// through a double-buffered int64 carry plane (read buffer rd, write rd^1),
// so no atomics and no cross-item ordering are needed.
#include "hk_internal.hpp"

namespace hk {

namespace {

__device__ __forceinline__ int32_t balanced29(int64_t v) {
  return (int32_t)(((v + (int64_t(1) << 28)) & (RADIX - 1)) - (int64_t(1) << 28));
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__global__ void k_fill32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill64(int64_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// A_rc = X_{r+c} - [r = c] xs  (diagonal shift first, as in determinant());
// carries of column c cleared.  One workgroup per column.
__global__ void __launch_bounds__(256) k_expand(const ColInfo* __restrict__ cols, int N, int WX,
                                                const int32_t* __restrict__ X,
                                                const int32_t* __restrict__ xs,
                                                int32_t* __restrict__ A, int64_t* __restrict__ Kc) {
  const int c = blockIdx.x;
  const ColInfo cc = cols[c];
  const int64_t n = (int64_t)cc.W * cc.R;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    int s = (int)(i / cc.R), lr = (int)(i - (int64_t)s * cc.R);
    int r = c + lr;
    int32_t v = 0;
    if (r < N && s < WX) {
      v = X[(int64_t)(r + c) * WX + s];
      if (lr == 0) v -= xs[s];
    }
    A[cc.aoff + i] = v;
  }
  const int64_t nk = (int64_t)2 * cc.nb * cc.R;
  for (int64_t i = threadIdx.x; i < nk; i += blockDim.x) Kc[cc.koff + i] = 0;
}

// acc[m] += sum_t C[t] * w(m - t), w(e) = hi[e] (e >= 0) or lo[16 + e] (e < 0)
__device__ __forceinline__ void mac_block(int64_t* acc, const int32_t* Cd, const int32_t* lo,
                                          const int32_t* hi) {
#pragma unroll
  for (int t = 0; t < WB; t++) {
#pragma unroll
    for (int m = 0; m < WB; m++) {
      const int e = m - t;
      const int32_t w = e >= 0 ? hi[e] : lo[WB + e];
      acc[m] += (int64_t)Cd[t] * (int64_t)w;
    }
  }
}

__device__ __forceinline__ void renorm(int64_t* acc) {
#pragma unroll
  for (int m = 0; m < WB; m++) {
    int64_t h = acc[m] >> DB;
    acc[m] -= h << DB;
    acc[m + 1] += h;
  }
}

// Rank-(k1-k0) update of columns [c_lo, c_hi):
//   A_rc -= sum_{k0 <= k < k1} C_k[c] L_k[r]      (exact)
// One wavefront per (column, 64-row tile, 16-digit output block).  C_k[c]
// digits are wavefront-uniform (scalar loads, SGPR operands of the MACs);
// L_k[r] digits are per lane and slide through a 31-digit register window.
__global__ void __launch_bounds__(256) k_update(const ColInfo* __restrict__ cols,
                                                const int32_t* __restrict__ itemStart,
                                                int32_t* __restrict__ A, int64_t* __restrict__ Kc,
                                                const int32_t* __restrict__ Cb,
                                                const int32_t* __restrict__ Lb,
                                                const int32_t* __restrict__ nCw,
                                                const int32_t* __restrict__ nLw,
                                                int32_t* __restrict__ flags, int N, int k0, int k1,
                                                int c_lo, int c_hi, int rd) {
  const int wave = uni(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int base = itemStart[c_lo];
  const int it = base + blockIdx.x * 4 + wave;
  if (it >= itemStart[c_hi]) return;
  int lo = c_lo, hi = c_hi - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (itemStart[mid] <= it) lo = mid; else hi = mid - 1;
  }
  const int c = uni(lo);
  const ColInfo cc = cols[c];
  const int rem = it - itemStart[c];
  const int T = cc.R >> 6;
  const int q = uni(rem / T);
  const int t = uni(rem - q * T);
  const int r = c + 64 * t + lane;
  const bool active = r < N;
  const int rr = active ? r : N - 1;

  int64_t acc[WB + 1];
#pragma unroll
  for (int m = 0; m <= WB; m++) acc[m] = 0;
  int cnt = 0;

  for (int k = k0; k < k1; k++) {
    const ColInfo kk = cols[k];
    const int nC = min(uni(nCw[tri_index(N, k, c)]), kk.CW - WB);
    const int nLl = active ? nLw[tri_index(N, k, rr)] : 0;
    const int nL = min(uni(wave_max(nLl)), kk.LW - 2 * WB);
    const int u_lo = max(0, q - (nC + WB - 1) / WB + 1);
    const int u_hi = min(q, (nL + WB - 2) / WB);
    if (nC == 0 || nL == 0 || u_lo > u_hi) continue;
    const int32_t* Cp = Cb + kk.coff + (int64_t)(c - k) * kk.CW;
    const int32_t* Lp = Lb + kk.loff + (rr - k);
    const int64_t P = kk.R;
    int32_t D[WB], U[WB], Cd[WB];
    if (u_lo == 0) {
#pragma unroll
      for (int e = 0; e < WB; e++) D[e] = 0;
    } else {
#pragma unroll
      for (int e = 0; e < WB; e++) D[e] = Lp[(int64_t)(WB * u_lo - WB + e) * P];
    }
    for (int u = u_lo; u <= u_hi; u += 2) {
#pragma unroll
      for (int e = 0; e < WB; e++) U[e] = Lp[(int64_t)(WB * u + e) * P];
      {
        const int32_t* cp = Cp + WB * (q - u);
#pragma unroll
        for (int e = 0; e < WB; e++) Cd[e] = cp[e];
      }
      mac_block(acc, Cd, D, U);
      cnt += WB;
      if (cnt >= 96) { renorm(acc); cnt = 0; }
      if (u + 1 > u_hi) break;
#pragma unroll
      for (int e = 0; e < WB; e++) D[e] = Lp[(int64_t)(WB * (u + 1) + e) * P];
      {
        const int32_t* cp = Cp + WB * (q - u - 1);
#pragma unroll
        for (int e = 0; e < WB; e++) Cd[e] = cp[e];
      }
      mac_block(acc, Cd, U, D);
      cnt += WB;
      if (cnt >= 96) { renorm(acc); cnt = 0; }
    }
  }
  if (!active) return;
  const int lr = r - c;
  int64_t* Kcol = Kc + cc.koff;
  int64_t v = 0;
  if (q > 0) v = Kcol[((int64_t)rd * cc.nb + q) * cc.R + lr];
  int32_t* Ap = A + cc.aoff + (int64_t)(WB * q) * cc.R + lr;
#pragma unroll
  for (int m = 0; m < WB; m++) {
    v += (int64_t)Ap[(int64_t)m * cc.R] - acc[m];
    const int32_t d = balanced29(v);
    Ap[(int64_t)m * cc.R] = d;
    v = (v - d) >> DB;
  }
  v -= acc[WB];
  if (q + 1 < cc.nb) Kcol[((int64_t)(rd ^ 1) * cc.nb + q + 1) * cc.R + lr] = v;
  else if (v != 0) atomicOr(&flags[0], 1);
}

// Column c after all its updates: normalise A_rc (folding pending block
// carries of buffer rd), C = RNE(A / 2^h), written as balanced digits (for
// the update) and as standard magnitude digits (for the division); the pivot
// row also stores |d| 2^sh normalised for the division.  One thread per row.
__global__ void __launch_bounds__(64) k_finalize(const ColInfo* __restrict__ cols, int N, int c,
                                                 int rd, int h, int32_t* __restrict__ A,
                                                 const int64_t* __restrict__ Kc,
                                                 int32_t* __restrict__ Cb, uint32_t* __restrict__ S,
                                                 uint32_t* __restrict__ Dd, int32_t* __restrict__ dinfo,
                                                 int32_t* __restrict__ nCw, int32_t* __restrict__ nCs,
                                                 int32_t* __restrict__ b32C, int32_t* __restrict__ flags) {
  const int r = c + blockIdx.x * 64 + threadIdx.x;
  if (r >= N) return;
  const ColInfo cc = cols[c];
  const int lr = r - c;
  const int W = cc.W;
  int32_t* Ap = A + cc.aoff + lr;
  const int64_t* Kcol = Kc + cc.koff;
  // pass 1: balanced normalisation in place
  int64_t v = 0;
  int top = -1;
  for (int s = 0; s < W; s++) {
    if (s > 0 && (s % WB) == 0) v += Kcol[((int64_t)rd * cc.nb + s / WB) * cc.R + lr];
    v += Ap[(int64_t)s * cc.R];
    const int32_t d = balanced29(v);
    Ap[(int64_t)s * cc.R] = d;
    v = (v - d) >> DB;
    if (d != 0) top = s;
  }
  if (v != 0) atomicOr(&flags[0], 2);
  const bool neg = top >= 0 && Ap[(int64_t)top * cc.R] < 0;
  // pass 2: |A| as standard digits, streamed through the RNE shift by h bits
  const int hq = h / DB, hb = h % DB;
  const int hbit_digit = (h - 1) / DB, hbit = (h - 1) % DB;
  int64_t bor = 0;              // carry while converting balanced -> standard
  int half = 0, sticky = 0;
  uint32_t prev = 0;            // standard digit s-1 (for the shifted output)
  int64_t rc = 0;               // RNE increment carry through the output
  int64_t bc = 0;               // balanced conversion carry of the output
  int nout = 0;
  const int64_t CW = cc.CW;
  int32_t* Crow = Cb + cc.coff + (int64_t)lr * CW;
  uint32_t* Srow = S + cc.soff + (int64_t)lr * CW;
  int ctop = -1, stop = -1;
  uint32_t stopv = 0;
  bool inc = false;
  auto emit = [&](uint32_t o) {
    // o: output standard digit before the RNE increment
    if (nout == 0) {
      inc = half && (sticky || (o & 1));
      rc = inc ? 1 : 0;
    }
    int64_t x = (int64_t)o + rc;
    uint32_t so = (uint32_t)(x & (RADIX - 1));
    rc = x >> DB;
    Srow[nout] = so;
    if (so) { stop = nout; stopv = so; }
    int64_t y = (int64_t)so + bc;
    if (y >= (int64_t(1) << 28)) { y -= RADIX; bc = 1; } else bc = 0;
    const int32_t bd = (int32_t)(neg ? -y : y);
    Crow[nout] = bd;
    if (bd) ctop = nout;
    nout++;
  };
  for (int s = 0; s <= W; s++) {
    uint32_t u = 0;
    if (s < W) {
      int64_t a = Ap[(int64_t)s * cc.R];
      int64_t x = (neg ? -a : a) + bor;
      u = (uint32_t)(x & (RADIX - 1));
      bor = x >> DB;
    }
    if (s == hbit_digit) {
      half = (u >> hbit) & 1;
      if (hbit > 0 && (u & ((1u << hbit) - 1))) sticky = 1;
    } else if (s < hbit_digit && u) {
      sticky = 1;
    }
    if (s > hq) emit((prev >> hb) | (hb ? ((u << (DB - hb)) & (uint32_t)(RADIX - 1)) : 0u));
    prev = u;
  }
  // flush: the increment carry and the balanced carry may add digits
  if (rc || bc) {
    int64_t x = rc;
    rc = 0;
    uint32_t so = (uint32_t)x;
    if (nout < CW) {
      Srow[nout] = so;
      if (so) { stop = nout; stopv = so; }
      int64_t y = (int64_t)so + bc;
      if (y >= (int64_t(1) << 28)) { y -= RADIX; bc = 1; } else bc = 0;
      const int32_t bd = (int32_t)(neg ? -y : y);
      Crow[nout] = bd;
      if (bd) ctop = nout;
      nout++;
    }
    if (bc && nout < CW) {
      Srow[nout] = 0;
      Crow[nout] = neg ? -1 : 1;
      ctop = nout;
      nout++;
    }
  }
  for (int i = nout; i < CW; i++) { Crow[i] = 0; Srow[i] = 0; }
  const int64_t ti = tri_index(N, c, r);
  nCw[ti] = ctop + 1;
  nCs[ti] = stop + 1;
  const int bits = stop < 0 ? 0 : DB * stop + (32 - __clz(stopv));
  b32C[ti] = (bits + 31) / 32;
  if (r == c) {
    // pivot: d_c = C_c[c]
    if (stop < 0 || neg) {
      atomicMin(&flags[1], c);
      if (stop >= 0 && neg) atomicAdd(&flags[2], 1);
    }
    if (stop >= 0) {
      // |d| shifted left so that its top digit has bit 28 set
      const int sh = 28 - (31 - __clz(stopv));
      uint32_t* Dp = Dd + cc.doff;
      uint32_t carry = 0;
      for (int i = 0; i <= stop; i++) {
        uint64_t x = ((uint64_t)Srow[i] << sh) | carry;
        Dp[i] = (uint32_t)(x & (RADIX - 1));
        carry = (uint32_t)(x >> DB);
      }
      dinfo[4 * c] = stop + 1;
      dinfo[4 * c + 1] = sh;
      dinfo[4 * c + 2] = neg ? 1 : 0;
    } else {
      dinfo[4 * c] = 0;
      dinfo[4 * c + 1] = 0;
      dinfo[4 * c + 2] = 0;
    }
  }
}

// L_c[r] = RNE(C_c[r] 2^h / d_c) for one row per 64-lane workgroup: schoolbook
// long division in radix 2^29 with a lazily normalised int64 remainder in
// LDS.  Each quotient digit is estimated from the top three remainder digits
// against the top three divisor digits in float64 (error < 1/2 + 2^-20), so
// quotient digits are signed and the remainder stays within (1/2 + eps) d;
// the final remainder decides the rounding (ties to even).
__global__ void __launch_bounds__(64) k_divide(const ColInfo* __restrict__ cols, int N, int c,
                                               int h, const uint32_t* __restrict__ S,
                                               const uint32_t* __restrict__ Dd,
                                               const int32_t* __restrict__ dinfo,
                                               const int32_t* __restrict__ Cb,
                                               const int32_t* __restrict__ nCs,
                                               int32_t* __restrict__ Lb, int32_t* __restrict__ nLw,
                                               int32_t* __restrict__ flags) {
  extern __shared__ int64_t smem[];
  const int r = c + 1 + blockIdx.x;
  const int lane = threadIdx.x;
  const ColInfo cc = cols[c];
  const int nd = dinfo[4 * c], sh = dinfo[4 * c + 1], negd = dinfo[4 * c + 2];
  const int64_t ti = tri_index(N, c, r);
  const int ns = nCs[ti];
  const int lr = r - c;
  int32_t* Lp = Lb + cc.loff + lr;
  const int64_t P = cc.R;
  const int LW = cc.LW;
  // sign of C_c[r]: top balanced digit
  const int32_t* Crow = Cb + cc.coff + (int64_t)lr * cc.CW;
  if (nd == 0) {  // zero pivot: nothing to divide by
    for (int j = lane; j < LW; j += 64) Lp[(int64_t)j * P] = 0;
    if (lane == 0) { nLw[ti] = 0; atomicOr(&flags[0], 4); }
    return;
  }
  const int Sbits = h + sh, Sq = Sbits / DB, Sb = Sbits % DB;
  const int nu = ns == 0 ? 0 : Sq + ns + 1;
  if (nu < nd) {  // quotient below 2/2^29: rounds to zero
    for (int j = lane; j < LW; j += 64) Lp[(int64_t)j * P] = 0;
    if (lane == 0) nLw[ti] = 0;
    return;
  }
  int64_t* rem = smem;                       // nu + 3
  int64_t* dd = rem + (nu + 3);              // nd + 1 (dd[nd] = 0)
  int64_t* qd = dd + (nd + 1);               // nu - nd + 2
  __shared__ int64_t qslot;
  __shared__ int negC;
  const uint32_t* Srow = S + cc.soff + (int64_t)lr * cc.CW;
  const uint32_t* Dp = Dd + cc.doff;
  for (int i = lane; i <= nd; i += 64) dd[i] = i < nd ? (int64_t)Dp[i] : 0;
  for (int s = lane; s < nu + 3; s += 64) {
    int64_t x = 0;
    if (s >= Sq && s < nu) {
      const int i = s - Sq;  // source digit index of the shifted value
      uint64_t a = i < ns ? (uint64_t)Srow[i] : 0;
      uint64_t b = (i >= 1 && i - 1 < ns) ? (uint64_t)Srow[i - 1] : 0;
      x = (int64_t)(((a << Sb) | (Sb ? (b >> (DB - Sb)) : 0)) & (RADIX - 1));
    }
    rem[s] = x;
  }
  if (lane == 0) {
    int t = -1;
    for (int i = cc.CW - 1; i >= 0; i--) if (Crow[i] != 0) { t = i; break; }
    negC = (t >= 0 && Crow[t] < 0) ? 1 : 0;
  }
  const int jmax = nu - nd;
  for (int j = lane; j <= jmax + 1; j += 64) qd[j] = 0;
  __syncthreads();
  const double R = (double)RADIX;
  const double D3 = (double)dd[nd - 1] * R * R + (nd >= 2 ? (double)dd[nd - 2] * R : 0.0) +
                    (nd >= 3 ? (double)dd[nd - 3] : 0.0);
  int since = 0;
  for (int j = jmax; j >= 0; j--) {
    if (lane == 0) {
      const int t = j + nd;
      rem[t] += rem[t + 1] << DB;
      rem[t + 1] = 0;
      for (int s = t - 2; s < t; s++) {
        if (s < 0) continue;
        int64_t cy = rem[s] >> DB;
        rem[s] -= cy << DB;
        rem[s + 1] += cy;
      }
      const double T = (double)rem[t] * R * R + (t >= 1 ? (double)rem[t - 1] * R : 0.0) +
                       (t >= 2 ? (double)rem[t - 2] : 0.0);
      const int64_t qq = (int64_t)rint(T * R / D3);
      qd[j] = qq;
      qslot = qq;
    }
    __syncthreads();
    const int64_t qq = qslot;
    if (qq != 0)
      for (int i = lane; i < nd; i += 64) rem[j + i] -= qq * dd[i];
    __syncthreads();
    if (++since == 12) {
      since = 0;
      for (int s = j + lane; s < j + nd - 1; s += 64) {
        const int64_t x = rem[s];
        const int64_t cy = x >> DB;
        if (cy) {
          atomicAdd((unsigned long long*)&rem[s], (unsigned long long)(-(cy << DB)));
          atomicAdd((unsigned long long*)&rem[s + 1], (unsigned long long)cy);
        }
      }
      __syncthreads();
    }
  }
  // rounding decision from the final remainder Rem = window [0, nd]
  if (lane == 0) {
    rem[nd] += rem[nd + 1] << DB;
    rem[nd + 1] = 0;
    for (int s = nd - 2; s < nd; s++) {
      if (s < 0) continue;
      int64_t cy = rem[s] >> DB;
      rem[s] -= cy << DB;
      rem[s + 1] += cy;
    }
    const double T = (double)rem[nd] * R * R + (nd >= 1 ? (double)rem[nd - 1] * R : 0.0) +
                     (nd >= 2 ? (double)rem[nd - 2] : 0.0);
    const double f = T * R / D3;   // Rem / d'
    int adj = 0;
    const double af = fabs(f);
    if (fabs(2.0 * af - 1.0) > 1e-6) {
      adj = af > 0.5 ? (f > 0 ? 1 : -1) : 0;
    } else {
      // exact comparison of 2 Rem with +d' and -d'
      int64_t v1 = 0, v2 = 0;
      int nz1 = 0, nz2 = 0;
      for (int s = 0; s <= nd + 1; s++) {
        const int64_t twor = 2 * rem[s];
        v1 += twor - dd[s <= nd ? s : nd];
        v2 += twor + dd[s <= nd ? s : nd];
        nz1 |= (v1 & (RADIX - 1)) != 0;
        nz2 |= (v2 & (RADIX - 1)) != 0;
        v1 >>= DB;
        v2 >>= DB;
      }
      const int s1 = v1 < 0 ? -1 : ((v1 == 0 && !nz1) ? 0 : 1);
      const int s2 = v2 < 0 ? -1 : ((v2 == 0 && !nz2) ? 0 : 1);
      const int odd = (int)(qd[0] & 1);
      if (s1 > 0) adj = 1;
      else if (s1 == 0) adj = odd ? 1 : 0;
      else if (s2 < 0) adj = -1;
      else if (s2 == 0) adj = odd ? -1 : 0;
    }
    qd[0] += adj;
  }
  __syncthreads();
  // quotient digits -> balanced digits (one carry step suffices: |q| <= 2^30)
  const int nq = jmax + 2;
  int mytop = -1;
  const int sgn = (negC ^ negd) ? -1 : 1;
  for (int j = lane; j < LW; j += 64) {
    int64_t out = 0;
    if (j < nq) {
      const int64_t x = j <= jmax ? qd[j] : 0;
      out = balanced29(x);
      if (j >= 1 && j - 1 <= jmax) {
        const int64_t y = qd[j - 1];
        out += (y - balanced29(y)) >> DB;
      }
    }
    const int32_t o = (int32_t)(sgn * out);
    Lp[(int64_t)j * P] = o;
    if (o != 0) mytop = j;
  }
  const int t = wave_max(mytop);
  if (lane == 0) {
    nLw[ti] = t + 1;
    if (t + 1 > LW - 32) atomicOr(&flags[0], 8);
  }
}

// exact ceil(bits/32) of every L entry (for the algorithmic work count)
__global__ void k_bitsL(const ColInfo* __restrict__ cols, int N, const int32_t* __restrict__ Lb,
                        const int32_t* __restrict__ nLw, int32_t* __restrict__ b32L) {
  const int64_t ntri = (int64_t)N * (N + 1) / 2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntri;
       i += (int64_t)gridDim.x * blockDim.x) {
    // recover (k, r) from the triangle index
    int k = (int)((2.0 * N + 1 - sqrt((2.0 * N + 1) * (2.0 * N + 1) - 8.0 * (double)i)) / 2);
    while (k > 0 && tri_index(N, k, k) > i) k--;
    while (k + 1 < N && tri_index(N, k + 1, k + 1) <= i) k++;
    const int r = k + (int)(i - tri_index(N, k, k));
    if (r == k) { b32L[i] = 0; continue; }
    const ColInfo kk = cols[k];
    const int n = nLw[i];
    const int32_t* Lp = Lb + kk.loff + (r - k);
    int negv = 0;
    for (int j = n - 1; j >= 0; j--) {
      const int32_t d = Lp[(int64_t)j * kk.R];
      if (d) { negv = d < 0; break; }
    }
    int64_t bor = 0;
    int top = -1;
    uint32_t topv = 0;
    for (int j = 0; j < n; j++) {
      const int64_t a = Lp[(int64_t)j * kk.R];
      const int64_t x = (negv ? -a : a) + bor;
      const uint32_t u = (uint32_t)(x & (RADIX - 1));
      bor = x >> DB;
      if (u) { top = j; topv = u; }
    }
    const int bits = top < 0 ? 0 : DB * top + (32 - __clz(topv));
    b32L[i] = (bits + 31) / 32;
  }
}

// pivots d_k = C_k[k] gathered into one buffer of N rows x ld digits
__global__ void k_gather_pivots(const ColInfo* __restrict__ cols, int N, int ld,
                                const int32_t* __restrict__ Cb, int32_t* __restrict__ out) {
  const int k = blockIdx.x;
  const ColInfo kk = cols[k];
  for (int i = threadIdx.x; i < ld; i += blockDim.x)
    out[(int64_t)k * ld + i] = i < kk.CW ? Cb[kk.coff + i] : 0;
}

int blocks_for(int64_t n, int tpb) {
  int64_t b = (n + tpb - 1) / tpb;
  if (b > 65535) b = 65535;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

hipError_t launch_fill32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill64(int64_t* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_expand(const Plan& P, const DevPtrs& D, hipStream_t s) {
  hipLaunchKernelGGL(k_expand, dim3(P.N), dim3(256), 0, s, D.cols, P.N, P.WX, D.X, D.xs, D.A, D.Kc);
  return hipGetLastError();
}
hipError_t launch_update(const Plan& P, const DevPtrs& D, int k0, int k1, int c_lo, int c_hi,
                         int rd, hipStream_t s) {
  const int64_t items = (int64_t)P.itemStart[c_hi] - P.itemStart[c_lo];
  if (items <= 0) return hipSuccess;
  const int blocks = (int)((items + 3) / 4);
  hipLaunchKernelGGL(k_update, dim3(blocks), dim3(256), 0, s, D.cols, D.itemStart, D.A, D.Kc,
                     D.C, D.L, D.nC, D.nL, D.flags, P.N, k0, k1, c_lo, c_hi, rd);
  return hipGetLastError();
}
hipError_t launch_finalize(const Plan& P, const DevPtrs& D, int c, int rd, hipStream_t s) {
  const int rows = P.N - c;
  hipLaunchKernelGGL(k_finalize, dim3((rows + 63) / 64), dim3(64), 0, s, D.cols, P.N, c, rd, P.h,
                     D.A, D.Kc, D.C, D.S, D.D, D.dinfo, D.nC, D.nCs, D.b32C, D.flags);
  return hipGetLastError();
}
hipError_t launch_divide(const Plan& P, const DevPtrs& D, int c, hipStream_t s) {
  const int rows = P.N - c - 1;
  if (rows <= 0) return hipSuccess;
  const ColInfo& cc = P.cols[c];
  // rem: nu + 3 with nu <= Sq + CW + 1; dd: W + 2; qd: nu + 2
  const int Sq = (P.h + 28) / DB + 1;
  const int nu_max = Sq + cc.CW + 1;
  const size_t shm = sizeof(int64_t) * (size_t)((nu_max + 3) + (cc.W + 3) + (nu_max + 3));
  hipLaunchKernelGGL(k_divide, dim3(rows), dim3(64), shm, s, D.cols, P.N, c, P.h, D.S, D.D,
                     D.dinfo, D.C, D.nCs, D.L, D.nL, D.flags);
  return hipGetLastError();
}
hipError_t launch_gather_pivots(const Plan& P, const DevPtrs& D, int32_t* out, int ld,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_gather_pivots, dim3(P.N), dim3(64), 0, s, D.cols, P.N, ld, D.C, out);
  return hipGetLastError();
}
hipError_t launch_bits(const Plan& P, const DevPtrs& D, hipStream_t s) {
  hipLaunchKernelGGL(k_bitsL, dim3(blocks_for(P.ntri, 256)), dim3(256), 0, s, D.cols, P.N, D.L,
                     D.nL, D.b32L);
  return hipGetLastError();
}

}  // namespace hk
