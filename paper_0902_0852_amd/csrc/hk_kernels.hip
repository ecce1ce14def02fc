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
#include <climits>
#include <hip/hip_ext.h>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "hk_internal.hpp"

namespace hk {

namespace {

__device__ __forceinline__ int32_t balanced29(int64_t v) {
  return (int32_t)(((v + (int64_t(1) << 28)) & (RADIX - 1)) - (int64_t(1) << 28));
}

// A balanced radix-2^29 digit d (|d| <= 2^28) as four signed bytes,
// d = b0 + b1 2^8 + b2 2^16 + b3 2^24 with b0, b1, b2 in [-128, 127] and
// |b3| <= 16: the operands of the matrix-core update.
__device__ __forceinline__ void split_bytes(int32_t d, int32_t& b0, int32_t& b1, int32_t& b2, int32_t& b3) {
  b0 = (d << 24) >> 24;
  d = (d - b0) >> 8;
  b1 = (d << 24) >> 24;
  d = (d - b1) >> 8;
  b2 = (d << 24) >> 24;
  b3 = (d - b2) >> 8;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// wave_max for values that are -1 or increase with the lane among the lanes
// where they are not: the value of the highest such lane (one ballot and one
// lane read instead of six cross-lane shuffles)
__device__ __forceinline__ int wave_max_mono(int v) {
  const uint64_t m = __ballot(v >= 0);
  return m == 0 ? -1 : __builtin_amdgcn_readlane(v, 63 - __clzll((long long)m));
}

// wave_max for v = -1 or lane + 64 k (a lane's last index of a loop over
// j = lane, lane + 64, ...; k <= kmax): the highest k that any lane reached,
// then the highest such lane, by ballots
__device__ __forceinline__ int wave_max_strided(int v, int kmax) {
  const int lane = threadIdx.x & 63;
  const int k = v >= 0 ? (v - lane) >> 6 : -1;
  for (int kk = kmax; kk >= 0; kk--) {
    const uint64_t m = __ballot(k == kk);
    if (m) return 64 * kk + 63 - __clzll((long long)m);
  }
  return -1;
}

// Device memory through global-address-space pointers: loads and stores
// become global_* instructions, which the compiler never has to order against
// LDS traffic (flat ones count against the LDS wait counter as well).
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* gp(T* p) { return (GLOBAL T*)p; }
__device__ __forceinline__ void gor(GLOBAL int32_t* f, int32_t v) {
  __hip_atomic_fetch_or(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// An empty asm statement that takes v in a register: loads issued before it
// cannot be sunk by the compiler into a branch of their own (each followed by
// a wait) when their value is masked afterwards; a batch of loads from
// clamped indices, pinned, then masked, costs one LDS round trip.
template <typename T>
__device__ __forceinline__ void pin(T& v) { asm volatile("" : "+v"(v)); }

// 64-bit lane moves: the value of lane i - 1 (lane 0: 0) by a DPP wave
// shift, and the value of one (uniform) lane
__device__ __forceinline__ int64_t lane_shr1(int64_t v) {
  const int32_t lo = __builtin_amdgcn_update_dpp(0, (int32_t)v, 0x138, 0xf, 0xf, false);
  const int32_t hi = __builtin_amdgcn_update_dpp(0, (int32_t)(v >> 32), 0x138, 0xf, 0xf, false);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int64_t lane_read(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}


// wavefront-uniform operand digits are read through the constant address
// space so that they arrive by scalar loads into SGPRs
typedef const __attribute__((address_space(4))) int32_t cint32_t;

// a pointer every lane holds the same value of, moved into SGPRs
template <typename T>
__device__ __forceinline__ T* uptr(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}
// a read-only object at a wavefront-uniform address, by scalar loads
template <typename T>
__device__ __forceinline__ T sload(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  typedef const __attribute__((address_space(4))) uint32_t cword;
  const cword* q = (const cword*)uptr(p);
  union { T t; uint32_t w[sizeof(T) / 4]; } u;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); i++) u.w[i] = q[i];
  return u.t;
}

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
// carries of column c cleared.  One workgroup per (column, instance).
__global__ void __launch_bounds__(256) k_expand(const InstDesc* __restrict__ desc) {
  const InstDesc I = desc[blockIdx.y];
  const int c = blockIdx.x;
  if (!I.active || c >= I.N) return;
  const ColInfo cc = I.cols[c];
  const int64_t n = (int64_t)cc.W * cc.R;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    int s = (int)(i / cc.R), lr = (int)(i - (int64_t)s * cc.R);
    int r = c + lr;
    int32_t v = 0;
    if (r < I.N && s < I.WX) {
      v = I.X[(int64_t)(r + c) * I.WX + s];
      if (lr == 0) v -= I.xs[s];
    }
    I.A[cc.aoff + i] = v;
  }
  const int64_t nk = (int64_t)2 * cc.nb * cc.R;
  for (int64_t i = threadIdx.x; i < nk; i += blockDim.x) I.Kc[cc.koff + i] = 0;
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

// Accumulate sum_{k} C_k * L_k into the 16 output columns of block q:
// C_k (uniform: wavefront-shared digits Cp[0..nC), zero padded to a multiple
// of 16) times L_k (per lane: digit j at Lbase[j * P + lo], zero padded by
// >= 30 digits), product scanning through a 31-digit sliding register window.
// L digits come by buffer loads: the digit-plane offset j P is a scalar
// operand, the lane offset lo a vector one, and the region size bounds every
// access (a load outside it returns 0).
__device__ __forceinline__ void accum_block(int64_t* acc, int& cnt, const int32_t* Cp, int nC,
                                            const int32_t* Lbase, int64_t nbytes, int lo, int P,
                                            int nL, int q) {
  const int u_lo = max(0, q - (nC + WB - 1) / WB + 1);
  const int u_hi = min(q, (nL + WB - 2) / WB);
  if (nC <= 0 || nL <= 0 || u_lo > u_hi) return;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)Lbase, (short)0, (int)min(nbytes, (int64_t)0x7fffffff), 0x00020000);
  const int vo = lo * 4;
  const int pb = P * 4;
  int32_t D[WB], U[WB], Cd[WB];
  if (u_lo == 0) {
#pragma unroll
    for (int e = 0; e < WB; e++) D[e] = 0;
  } else {
#pragma unroll
    for (int e = 0; e < WB; e++)
      D[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, (WB * u_lo - WB + e) * pb, 0);
  }
  for (int u = u_lo; u <= u_hi; u += 2) {
#pragma unroll
    for (int e = 0; e < WB; e++) U[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, (WB * u + e) * pb, 0);
    {
      const cint32_t* cp = (const cint32_t*)(Cp + WB * (q - u));
#pragma unroll
      for (int e = 0; e < WB; e++) Cd[e] = cp[e];
    }
    mac_block(acc, Cd, D, U);
    cnt += WB;
    if (cnt >= 96) { renorm(acc); cnt = 0; }
    if (u + 1 > u_hi) break;
#pragma unroll
    for (int e = 0; e < WB; e++)
      D[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, (WB * (u + 1) + e) * pb, 0);
    {
      const cint32_t* cp = (const cint32_t*)(Cp + WB * (q - u - 1));
#pragma unroll
      for (int e = 0; e < WB; e++) Cd[e] = cp[e];
    }
    mac_block(acc, Cd, U, D);
    cnt += WB;
    if (cnt >= 96) { renorm(acc); cnt = 0; }
  }
}

// A's 16 digits of block q -= acc, with the pending carry into this block
// (kin, NULL for block 0) folded in; the carry out goes to kout (NULL for the
// top block, where it must vanish).  The digits are addressed as in the
// multiply loop: a buffer descriptor over the column's digit planes (Acol,
// abytes), the lane's row as the vector offset and the digit plane as a
// scalar offset, so no 64-bit address is held per digit.  All 16 digits
// (and the carry) are loaded before the first store, so the loads are in
// flight together rather than one after another.
__device__ __forceinline__ void apply_block(const int64_t* acc, const int32_t* Acol, int64_t abytes, int lr,
                                            int R, int q, const GLOBAL int64_t* kin, GLOBAL int64_t* kout,
                                            GLOBAL int32_t* flags) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)Acol, (short)0, (int)min(abytes, (int64_t)0x7fffffff), 0x00020000);
  const int vo = lr * 4;
  const int pb = R * 4;
  const int sb = WB * q * pb;
  int32_t a[WB];
#pragma unroll
  for (int m = 0; m < WB; m++) a[m] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, sb + m * pb, 0);
  int64_t v = kin ? *kin : 0;
#pragma unroll
  for (int m = 0; m < WB; m++) {
    v += (int64_t)a[m] - acc[m];
    const int32_t d = balanced29(v);
    __builtin_amdgcn_raw_buffer_store_b32(d, rs, vo, sb + m * pb, 0);
    v = (v - d) >> DB;
  }
  v -= acc[WB];
  if (kout) *kout = v;
  else if (v != 0) gor(flags, 1);
}

// column and panel ranges of one update launch for an instance of size N:
// j = 0 trailing (columns [pc+bb, N), k in [pc, pc+bb)), j > 0 in-panel
// (column pc+j, k in [pc, pc+j)); false if the instance has nothing to do
__host__ __device__ inline bool update_range(int N, int pc, int b, int j, int& k0, int& k1, int& c_lo,
                                            int& c_hi) {
  if (j > 0) {
    if (pc + j >= N) return false;
    k0 = pc; k1 = pc + j; c_lo = pc + j; c_hi = pc + j + 1;
    return true;
  }
  const int bb = min(b, N - pc);
  if (bb <= 0 || pc + bb >= N) return false;
  k0 = pc; k1 = pc + bb;
  if (j == UPD_NEAR) { c_lo = pc + bb; c_hi = min(N, pc + 2 * bb); }
  else if (j == UPD_FAR) { c_lo = min(N, pc + 2 * bb); c_hi = N; }
  else { c_lo = pc + bb; c_hi = N; }
  return c_lo < c_hi;
}

// Rank-(k1-k0) update of the columns [c_lo, c_hi) of every instance:
//   A_rc -= sum_{k0 <= k < k1} C_k[c] L_k[r]      (exact)
// One wavefront per (instance, column, 64-row tile, 16-digit output block).
// C_k[c] digits are wavefront-uniform; L_k[r] digits are per lane.
// One item (wavefront), numbered `it` across the columns and instances of
// the launch.
// The instance, panel range [k0, k1), column c and the item's rank within
// its column (rem) of update item `it` of a launch; false if there is none or
// the instance is finished.  Wavefront-uniform.
__device__ __forceinline__ bool find_update_item(const InstDesc* __restrict__ desc, int count, int pc, int b,
                                                 int j, int it, int& inst, int& k0, int& k1, int& c, int& rem) {
  const int lane = threadIdx.x & 63;
  int c_lo = 0, c_hi = 0;
  inst = -1;
  for (int i = 0; i < count; i++) {
    int a0, a1, b0, b1;
    const int Ni = sload(&desc[i].N);
    if (!update_range(Ni, pc, b, j, a0, a1, b0, b1)) continue;
    const int32_t* is = sload(&desc[i].itemStart);
    const int n = sload(is + b1) - sload(is + b0);
    if (it < n) { inst = i; k0 = a0; k1 = a1; c_lo = b0; c_hi = b1; break; }
    it -= n;
  }
  inst = uni(inst);
  if (inst < 0) return false;
  const InstDesc I = sload(desc + inst);
  if (!I.active) return false;
  it += sload(I.itemStart + c_lo);
  // the column of the item: the last c in [c_lo, c_hi) with itemStart[c] <= it
  // (itemStart is nondecreasing), found by the whole wavefront reading 64
  // evenly spaced starts at once and narrowing to the interval the ballot
  // picks: one round for up to 64 columns, two up to 4096
  int lo = c_lo, n = c_hi - c_lo, start = 0;
  while (n > 1) {
    const int step = (n + 63) / 64;
    const int k = lane * step;
    const int v = k < n ? gp(I.itemStart)[lo + k] : INT_MAX;
    const uint64_t m = __ballot(v <= it);
    const int last = 63 - __clzll((long long)m);
    lo = uni(lo + last * step);
    n = min(step, c_hi - lo);
  }
  c = uni(lo);
  start = sload(I.itemStart + c);
  rem = it - start;
  return true;
}

__device__ __forceinline__ void update_item(const InstDesc* __restrict__ desc, int count, int pc, int b, int j,
                                            int rd, int it) {
  const int lane = threadIdx.x & 63;
  int inst, k0, k1, c, rem;
  if (!find_update_item(desc, count, pc, b, j, it, inst, k0, k1, c, rem)) return;
  const InstDesc I = sload(desc + inst);
  const int N = I.N;
  const ColInfo cc = sload(I.cols + c);
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
    const ColInfo kk = sload(I.cols + k);
    const int nC = min(sload(I.nC + tri_index(N, k, c)), kk.CW - WB);
    const int nLl = active ? gp(I.nL)[tri_index(N, k, rr)] : 0;
    const int nL = min(uni(wave_max(nLl)), kk.LW - 2 * WB);
    accum_block(acc, cnt, uptr(I.C + kk.coff + (int64_t)(c - k) * kk.CW), nC, uptr(I.L + kk.loff),
                (int64_t)kk.LW * kk.R * 4, rr - k, kk.R, nL, q);
  }
  if (!active) return;
  const int lr = r - c;
  int64_t* Kcol = I.Kc + cc.koff;
  apply_block(acc, uptr(I.A + cc.aoff), (int64_t)cc.W * cc.R * 4, lr, cc.R, q,
              q > 0 ? gp(Kcol + ((int64_t)rd * cc.nb + q) * cc.R + lr) : nullptr,
              q + 1 < cc.nb ? gp(Kcol + ((int64_t)(rd ^ 1) * cc.nb + q + 1) * cc.R + lr) : nullptr, gp(I.flags));
}

// The bulk of the update work: the trailing update of a panel (j = 0), or
// its columns beyond the next panel (UPD_FAR, look-ahead).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) k_update(const InstDesc* __restrict__ desc, int count, int pc,
                                                int b, int j, int rd) {
  update_item(desc, count, pc, b, j, rd, blockIdx.x * (blockDim.x >> 6) + uni(threadIdx.x >> 6));
}
// The small launches on the critical path: the in-panel updates (j > 0) and
// the next panel's columns (UPD_NEAR, look-ahead); the same items under a
// symbol of their own, so that they time and profile apart from the bulk.
// Their waves take the SIMDs' issue slots ahead of the bulk launch's waves
// that share them (the bulk only needs to finish before the panel after
// next), as the row waves of the column kernels do.
__global__ void __launch_bounds__(256) k_update_near(const InstDesc* __restrict__ desc, int count, int pc,
                                                     int b, int j, int rd) {
  __builtin_amdgcn_s_setprio(3);
  update_item(desc, count, pc, b, j, rd, blockIdx.x * (blockDim.x >> 6) + uni(threadIdx.x >> 6));
}

// ---------------------------------------------------------------------------
// The trailing update on the matrix cores.  Every digit of C and L splits
// exactly into four signed bytes (split_bytes), so the exact sum of digit
// products at output position t of an entry,
//   V_t = sum_{i + j = t} C_i L_j = sum_s 2^(8 s) D_s[t],
//   D_s[t] = sum_{p + q = s} sum_j c_p[t - j] l_q[j],
// is sixteen int8 products accumulated into seven int32 planes D_0..D_6.
// For one column c, 32 output positions t0 + i and 32 rows r, each D_s is a
// matrix product: a Toeplitz matrix of C's bytes (rows t, columns j, entry
// c_p[t - j], the same for every row r) times L's bytes (rows j, columns r),
// which is what v_mfma_i32_32x32x32_i8 computes, 32 digits j at a time.
// Products are accumulated over the panel's columns k in int32 (the host
// keeps sum_k nC_k below 2^15, so |D_s| < 4 2^14 2^15 = 2^31), then turned
// into 29-bit digits and carries and subtracted from A as in apply_block.

typedef int v16i __attribute__((ext_vector_type(16)));
typedef int v4i __attribute__((ext_vector_type(4)));

// bytes of one C byte plane in LDS for columns of at most Wm digits: the
// plane is stored reversed, byte y holding c_p[Wm + 64 - y], with 64 zero
// digits beyond both ends of C and a dword of slack for the aligned reads
__host__ __device__ inline int mma_plane_bytes(int Wm) { return (Wm + 140 + 15) / 16 * 16; }

// 16 bytes of a plane from byte y0 on (any alignment): five aligned dword
// reads and four byte-aligns
__device__ __forceinline__ v4i lds_bytes16(const uint32_t* plane, int y0) {
  const uint32_t* w = plane + (y0 >> 2);
  const uint32_t sh = (uint32_t)(y0 & 3);
  const uint32_t a0 = w[0], a1 = w[1], a2 = w[2], a3 = w[3], a4 = w[4];
  v4i r;
  r[0] = (int)__builtin_amdgcn_alignbyte(a1, a0, sh);
  r[1] = (int)__builtin_amdgcn_alignbyte(a2, a1, sh);
  r[2] = (int)__builtin_amdgcn_alignbyte(a3, a2, sh);
  r[3] = (int)__builtin_amdgcn_alignbyte(a4, a3, sh);
  return r;
}

// 64-bit value of lane l ^ 32
__device__ __forceinline__ int64_t swap_halves(int64_t v) {
  const int a = (((int)threadIdx.x & 63) ^ 32) << 2;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(a, (int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(a, (int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A's digits of block q (per lane) -= acc with the pending carry kin folded
// in and the carry out to kout, as apply_block, with the block offset a
// vector operand (the two halves of a wavefront apply different blocks)
__device__ __forceinline__ void apply_block_v(const int64_t* acc, const int32_t* Acol, int64_t abytes, int lr,
                                              int R, int q, const GLOBAL int64_t* kin, GLOBAL int64_t* kout,
                                              GLOBAL int32_t* flags) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)Acol, (short)0, (int)min(abytes, (int64_t)0x7fffffff), 0x00020000);
  const int pb = R * 4;
  const int vo = lr * 4 + WB * q * pb;
  int32_t a[WB];
#pragma unroll
  for (int m = 0; m < WB; m++) a[m] = __builtin_amdgcn_raw_buffer_load_b32(rs, vo, m * pb, 0);
  int64_t v = kin ? *kin : 0;
#pragma unroll
  for (int m = 0; m < WB; m++) {
    v += (int64_t)a[m] - acc[m];
    const int32_t d = balanced29(v);
    __builtin_amdgcn_raw_buffer_store_b32(d, rs, vo, m * pb, 0);
    v = (v - d) >> DB;
  }
  v -= acc[WB];
  if (kout) *kout = v;
  else if (v != 0) gor(flags, 1);
}

// The digits and carries of the tile's exact sums (from D) subtracted from
// A's blocks 2 q2 + h of row r (lane l: row r, half h = l / 32)
__device__ __forceinline__ void mma_apply(const v16i* D, const InstDesc& I, const ColInfo& cc, int c, int r,
                                          bool active, int q2, int rd, int lane) {
  const int h = lane >> 5;
  int32_t dg[16];
  int64_t cy[16];
#pragma unroll
  for (int v = 0; v < 16; v++) {
    const int64_t lo = (int64_t)D[0][v] + ((int64_t)D[1][v] << 8) + ((int64_t)D[2][v] << 16) +
                       ((int64_t)D[3][v] << 24);
    const int64_t hi = (int64_t)D[4][v] + ((int64_t)D[5][v] << 8) + ((int64_t)D[6][v] << 16);
    dg[v] = balanced29(lo);
    cy[v] = ((lo - dg[v]) >> DB) + (hi << 3);
  }
  int32_t rdg[8];
  int64_t rcy[8];
#pragma unroll
  for (int u = 0; u < 8; u++) {
    const int v = h ? u : u + 8;
    rdg[u] = (int32_t)swap_halves((int64_t)dg[v]);
    rcy[u] = swap_halves(cy[v]);
  }
  int64_t acc[WB + 1];
  int64_t prev = h ? cy[7] : 0;
#pragma unroll
  for (int m = 0; m < WB; m++) {
    const int grp = m >> 2, e = m & 3;
    const bool own = (grp & 1) == h;
    const int v = 8 * h + 4 * (grp >> 1) + e, u = 4 * (grp >> 1) + e;
    acc[m] = (int64_t)(own ? dg[v] : rdg[u]) + prev;
    prev = own ? cy[v] : rcy[u];
  }
  acc[WB] = h ? prev : 0;
  if (!active) return;
  const int lr = r - c, q = 2 * q2 + h;
  int64_t* Kcol = I.Kc + cc.koff;
  apply_block_v(acc, uptr(I.A + cc.aoff), (int64_t)cc.W * cc.R * 4, lr, cc.R, q,
                q > 0 ? gp(Kcol + ((int64_t)rd * cc.nb + q) * cc.R + lr) : nullptr,
                q + 1 < cc.nb ? gp(Kcol + ((int64_t)(rd ^ 1) * cc.nb + q + 1) * cc.R + lr) : nullptr,
                gp(I.flags));
}

// Where one item of the matrix-core update lies: column c, 32 rows (tile
// t32 of the column's 32-row tiles), output digits [32 q2, 32 q2 + 32)
// (blocks 2 q2 and 2 q2 + 1) of instance I.
struct MmaItem {
  InstDesc I;
  ColInfo cc;
  int k0, k1, c, q2, t32, r, rr;
  bool active;
};

// The item's digit products by the panel columns k0 + kf, k0 + kf + ks, ...
// into D (zeroed here).  Lane l: row r = c + 32 t32 + l % 32, half h = l / 32
// of the K operand digits.  lds: this wavefront's four C byte planes.
__device__ __forceinline__ void mma_accum(v16i* D, const MmaItem& T, int kf, int ks, int Wm, uint32_t* lds) {
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  const InstDesc& I = T.I;
  const int N = I.N, c = T.c, k0 = T.k0, k1 = T.k1, rr = T.rr;
  const bool active = T.active;
  const int t0 = 32 * T.q2;
  const int PB = mma_plane_bytes(Wm), X0 = Wm + 64;
  int8_t* planes = (int8_t*)lds;
#pragma unroll
  for (int s = 0; s < 7; s++)
#pragma unroll
    for (int v = 0; v < 16; v++) D[s][v] = 0;
  if (k0 + kf >= k1) return;
  // the digit counts of the next panel column are requested one column
  // ahead, and so are its first 512 digits of C (cvn, for column kpref)
  int nCn = sload(I.nC + tri_index(N, k0 + kf, c));
  int nLn = active ? gp(I.nL)[tri_index(N, k0 + kf, rr)] : 0;
  int32_t cvn[8];
  int kpref = -1;
  for (int k = k0 + kf; k < k1; k += ks) {
    const ColInfo kk = sload(I.cols + k);
    const int nC = min(nCn, kk.CW - WB);
    const int nLl = nLn;
    if (k + ks < k1) {
      nCn = sload(I.nC + tri_index(N, k + ks, c));
      nLn = active ? gp(I.nL)[tri_index(N, k + ks, rr)] : 0;
    }
    const int nL = min(uni(wave_max(nLl)), kk.LW - 2 * WB);
    const int jlo = max(0, t0 - nC + 1), jhi = min(nL, t0 + 32);
    if (nC <= 0 || jlo >= jhi) continue;
    const int g0 = jlo >> 5, g1 = (jhi - 1) >> 5;
    // L_k's byte planes of this lane's row (16 digits of each 32-digit
    // chunk) are loaded two chunks ahead of their products, C's Toeplitz
    // operands one chunk ahead, in three rotating register sets (no moves
    // between them, so no wait falls before its turn); the first two chunks
    // of L are requested before C's planes are built
    const GLOBAL int8_t* Lb = gp(I.L8 + kk.l8off + (int64_t)(rr - k) * 32 + 16 * h);
    const int64_t cs = (int64_t)kk.R * 32, ps = (int64_t)kk.G * cs;
    const int yb = X0 - t0 - i + 16 * h;
    v4i B0[4], B1[4], B2[4], A0[4], A1[4], A2[4];
    auto ldB = [&](v4i* Bx, int g) {
      const GLOBAL int8_t* p = Lb + min(g, g1) * cs;
#pragma unroll
      for (int q = 0; q < 4; q++) Bx[q] = *(const GLOBAL v4i*)(p + q * ps);
    };
    auto ldA = [&](v4i* Ax, int g) {
#pragma unroll
      for (int p = 0; p < 4; p++) Ax[p] = lds_bytes16(lds + p * (PB >> 2), yb + 32 * min(g, g1));
    };
    auto mm = [&](const v4i* Ax, const v4i* Bx) {
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int p = 0; p < 4; p++)
          D[p + q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Ax[p], Bx[q], D[p + q], 0, 0, 0);
    };
    ldB(B0, g0);
    ldB(B1, g0 + 1);
    // C_k[c] as four reversed byte planes, zero outside the digits
    for (int x = lane; x < PB; x += 64) lds[x] = 0;   // 4 planes of PB / 4 dwords
    {
      // C's digits in batches of 8 per lane, each batch's loads in flight
      // together (clamped indices, masked stores)
      const GLOBAL int32_t* Cg = gp(I.C + kk.coff + (int64_t)(c - k) * kk.CW);
      for (int x0 = 0; x0 < nC; x0 += 512) {
        int32_t cv[8];
        if (x0 == 0 && kpref == k) {
#pragma unroll
          for (int u = 0; u < 8; u++) cv[u] = cvn[u];
        } else {
#pragma unroll
          for (int u = 0; u < 8; u++) cv[u] = Cg[min(x0 + lane + 64 * u, nC - 1)];
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int x = x0 + lane + 64 * u;
          if (x < nC) {
            int32_t b0, b1, b2, b3;
            split_bytes(cv[u], b0, b1, b2, b3);
            const int y = X0 - x;
            planes[y] = (int8_t)b0;
            planes[PB + y] = (int8_t)b1;
            planes[2 * PB + y] = (int8_t)b2;
            planes[3 * PB + y] = (int8_t)b3;
          }
        }
      }
    }
    // the next panel column's first digits of C, in flight during this
    // column's products
    if (k + ks < k1) {
      const int kn = k + ks;
      const ColInfo kc = sload(I.cols + kn);
      const int nCx = min(nCn, kc.CW - WB);
      const GLOBAL int32_t* Cn = gp(I.C + kc.coff + (int64_t)(c - kn) * kc.CW);
#pragma unroll
      for (int u = 0; u < 8; u++) cvn[u] = Cn[min(lane + 64 * u, max(nCx - 1, 0))];
      kpref = kn;
    }
    ldA(A0, g0);
    for (int g = g0; g <= g1; g += 3) {
      ldB(B2, g + 2);
      ldA(A1, g + 1);
      mm(A0, B0);
      if (g + 1 > g1) break;
      ldB(B0, g + 3);
      ldA(A2, g + 2);
      mm(A1, B1);
      if (g + 2 > g1) break;
      ldB(B1, g + 4);
      ldA(A0, g + 3);
      mm(A2, B2);
    }
  }
}

// The item of update launch item `it`; false if there is none
__device__ __forceinline__ bool mma_find(const InstDesc* __restrict__ desc, int count, int pc, int b, int j, int it,
                                         MmaItem& T) {
  int inst, rem;
  if (!find_update_item(desc, count, pc, b, j, it, inst, T.k0, T.k1, T.c, rem)) return false;
  T.I = sload(desc + inst);
  T.cc = sload(T.I.cols + T.c);
  const int T32 = T.cc.R >> 5;
  T.q2 = uni(rem / T32);
  T.t32 = uni(rem - T.q2 * T32);
  T.r = T.c + 32 * T.t32 + (int)(threadIdx.x & 31);
  T.active = T.r < T.I.N;
  T.rr = T.active ? T.r : T.I.N - 1;
  return true;
}

// The digit products of one 32 x 32 tile on the matrix cores: D (zeroed
// here) accumulates the byte-plane products over the panel columns and
// their 32-digit chunks, with L's planes loaded two chunks ahead and C's
// Toeplitz operands one chunk ahead of their products (three rotating
// register sets, so no move between them makes a load wait before its turn).
// Per panel column kk of the workgroup (LDS): planes[kk] C's four byte
// planes, nCk[kk], nLk[kk] the digit counts, l8[kk] the byte offset of L's
// planes of the tile's first row, and csk/psk their chunk and plane strides.
struct MmaCols {
  const uint32_t* planes;   // nk sets of 4 planes of PB bytes
  const int* nCk;
  const int* nLk;
  const int64_t* l8;
  const int64_t* csk;
  const int64_t* psk;
  int nk, PB, X0;
};

__device__ __forceinline__ void mma_tile(v16i* D, const MmaCols& M, const GLOBAL int8_t* L8, int t0, int row,
                                         int lane) {
  const int i = lane & 31, h = lane >> 5;
#pragma unroll
  for (int s = 0; s < 7; s++)
#pragma unroll
    for (int v = 0; v < 16; v++) D[s][v] = 0;
  const int yb = M.X0 - t0 - i + 16 * h;
  for (int kk = 0; kk < M.nk; kk++) {
    const int nC = M.nCk[kk], nL = M.nLk[kk];
    const int jlo = max(0, t0 - nC + 1), jhi = min(nL, t0 + 32);
    if (nC <= 0 || jlo >= jhi) continue;
    const int g0 = jlo >> 5, g1 = (jhi - 1) >> 5;
    const GLOBAL int8_t* Lb = L8 + M.l8[kk] + (int64_t)row * 32 + 16 * h;
    const int64_t cs = M.csk[kk], ps = M.psk[kk];
    const uint32_t* pl = M.planes + kk * M.PB;     // 4 planes of PB / 4 dwords
    auto ldB = [&](v4i* Bx, int g) {
      const GLOBAL int8_t* p = Lb + min(g, g1) * cs;
#pragma unroll
      for (int q = 0; q < 4; q++) Bx[q] = *(const GLOBAL v4i*)(p + q * ps);
    };
    auto ldA = [&](v4i* Ax, int g) {
#pragma unroll
      for (int p = 0; p < 4; p++) Ax[p] = lds_bytes16(pl + p * (M.PB >> 2), yb + 32 * min(g, g1));
    };
    auto mm = [&](const v4i* Ax, const v4i* Bx) {
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int p = 0; p < 4; p++)
          D[p + q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Ax[p], Bx[q], D[p + q], 0, 0, 0);
    };
    v4i B0[4], B1[4], B2[4], A0[4], A1[4], A2[4];
    ldB(B0, g0);
    ldB(B1, g0 + 1);
    ldA(A0, g0);
    for (int g = g0; g <= g1; g += 3) {
      ldB(B2, g + 2);
      ldA(A1, g + 1);
      mm(A0, B0);
      if (g + 1 > g1) break;
      ldB(B0, g + 3);
      ldA(A2, g + 2);
      mm(A1, B1);
      if (g + 2 > g1) break;
      ldB(B1, g + 4);
      ldA(A0, g + 3);
      mm(A2, B2);
    }
  }
}

// The bulk update on the matrix cores, one workgroup per (instance, column,
// 32-row tile): its four wavefronts build C_k[c]'s byte planes of every panel
// column k once (LDS), then share out the column's 32-digit output tiles.
// Wm: the widest column of the launch; the LDS holds (k1 - k0) plane sets.
constexpr int MMA_RUN = 4;    // consecutive tiles per XCD turn (4, 16, 64, 256: 1712, 1732, 1829, 2174 ms per step)
constexpr int MMA_SPLIT_ITEMS = 512;   // near launches up to this many items: k_update_mma_sk

// Number of (32-row tile, column) pairs with rows in them of an instance of
// size N for the columns [c_lo, c_hi), tile t32 of column c covering rows
// c + 32 t32 .. c + 32 t32 + 31: for tile index t32 the columns below
// N - 32 t32.
__host__ __device__ inline int mma_tile_count(int N, int c_lo, int c_hi, int t32) {
  return max(0, min(c_hi, N - 32 * t32) - c_lo);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_update_mma(const InstDesc* __restrict__ desc, int count, int pc, int b,
                                                     int j, int rd, int Wm, int run) {
  extern __shared__ int64_t smem[];
  // the next panel's columns are on the critical path (as in k_update_mma_w)
  if (!update_is_bulk(j)) __builtin_amdgcn_s_setprio(3);
  const int lane = threadIdx.x & 63, w = uni(threadIdx.x >> 6), nw = blockDim.x >> 6;
  // Workgroups go round-robin to the chip's eight XCDs; each XCD takes runs
  // of `run` consecutive pairs, enumerated tile-major (for tile index 0,
  // every column, then tile index 1 ...), so that the workgroups one XCD
  // runs together read the same rows of L from its own L2, while the runs
  // alternate between the XCDs to spread the work evenly
  const int q = (int)(blockIdx.x >> 3);
  int it = ((q / run) * 8 + (int)(blockIdx.x & 7)) * run + q % run;
  int inst = -1, k0 = 0, k1 = 0, c_lo = 0, c_hi = 0;
  for (int i2 = 0; i2 < count; i2++) {
    int a0, a1, b0, b1;
    const int Ni = sload(&desc[i2].N);
    if (!update_range(Ni, pc, b, j, a0, a1, b0, b1)) continue;
    int n = 0;
    for (int t = 0; 32 * t < Ni - b0; t++) n += mma_tile_count(Ni, b0, b1, t);
    if (it < n) { inst = i2; k0 = a0; k1 = a1; c_lo = b0; c_hi = b1; break; }
    it -= n;
  }
  inst = uni(inst);
  if (inst < 0) return;
  const InstDesc I = sload(desc + inst);
  if (!I.active) return;
  const int N = I.N;
  int t32 = 0;
  for (;; t32++) {
    const int n = mma_tile_count(N, c_lo, c_hi, t32);
    if (it < n) break;
    it -= n;
  }
  t32 = uni(t32);
  const int c = uni(c_lo + it);
  const ColInfo cc = sload(I.cols + c);
  const int nk = k1 - k0;
  const int PB = mma_plane_bytes(Wm), X0 = Wm + 64;
  uint32_t* planes = (uint32_t*)smem;                       // nk x PB dwords
  int* nCk = (int*)(planes + nk * PB);
  int* nLk = nCk + nk;
  int64_t* l8 = (int64_t*)(((uintptr_t)(nLk + nk) + 7) & ~(uintptr_t)7);
  int64_t* csk = l8 + nk;
  int64_t* psk = csk + nk;
  const int i = lane & 31;
  const int r = c + 32 * t32 + i;
  const bool active = r < N;
  const int rr = active ? r : N - 1;
  // per panel column: digit counts (L's: the largest over the tile's rows)
  for (int kk = w; kk < nk; kk += nw) {
    const int k = k0 + kk;
    const ColInfo kc = sload(I.cols + k);
    const int nLl = active ? gp(I.nL)[tri_index(N, k, rr)] : 0;
    const int nL = min(uni(wave_max(nLl)), kc.LW - 2 * WB);
    if (lane == 0) {
      nCk[kk] = min(gp(I.nC)[tri_index(N, k, c)], kc.CW - WB);
      nLk[kk] = nL;
      l8[kk] = kc.l8off + (int64_t)(c + 32 * t32 - k) * 32;
      csk[kk] = (int64_t)kc.R * 32;
      psk[kk] = (int64_t)kc.G * kc.R * 32;
    }
  }
  for (int x = threadIdx.x; x < nk * PB; x += blockDim.x) planes[x] = 0;
  __syncthreads();
  // C_k[c] of every panel column as four reversed byte planes
  {
    int8_t* pb = (int8_t*)planes;
    for (int kk = 0; kk < nk; kk++) {
      const int k = k0 + kk;
      const ColInfo kc = sload(I.cols + k);
      const int nC = nCk[kk];
      const GLOBAL int32_t* Cg = gp(I.C + kc.coff + (int64_t)(c - k) * kc.CW);
      int8_t* pk = pb + (int64_t)kk * 4 * PB;
      for (int x0 = 0; x0 < nC; x0 += 4 * 256) {
        int32_t cv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) cv[u] = Cg[min(x0 + (int)threadIdx.x + (int)blockDim.x * u, max(nC - 1, 0))];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int x = x0 + threadIdx.x + blockDim.x * u;
          if (x < nC) {
            int32_t b0, b1, b2, b3;
            split_bytes(cv[u], b0, b1, b2, b3);
            const int y = X0 - x;
            pk[y] = (int8_t)b0;
            pk[PB + y] = (int8_t)b1;
            pk[2 * PB + y] = (int8_t)b2;
            pk[3 * PB + y] = (int8_t)b3;
          }
        }
      }
    }
  }
  __syncthreads();
  const MmaCols M{planes, nCk, nLk, l8, csk, psk, nk, PB, X0};
  const GLOBAL int8_t* L8 = gp(I.L8);
  v16i D[7];
  for (int q2 = w; q2 < (cc.nb >> 1); q2 += nw) {
    mma_tile(D, M, L8, 32 * q2, rr - (c + 32 * t32), lane);
    mma_apply(D, I, cc, c, r, active, q2, rd, lane);
  }
}
__host__ inline size_t mma_lds(int Wm, int nk) {
  return (size_t)nk * 4 * mma_plane_bytes(Wm) + 8 * (size_t)nk + 8 + 24 * (size_t)nk;
}

// The update on the matrix cores, one item per wavefront: the near launches
// with many items, and the bulk where the panel's C planes do not fit one
// workgroup's LDS.  Wm: the widest column of the launch (LDS: four C byte
// planes per wavefront).
__global__ void __launch_bounds__(256) k_update_mma_w(const InstDesc* __restrict__ desc, int count, int pc, int b,
                                                    int j, int rd, int Wm) {
  extern __shared__ int64_t smem[];
  const int w = uni(threadIdx.x >> 6);
  uint32_t* lds = (uint32_t*)smem + w * mma_plane_bytes(Wm);
  if (!update_is_bulk(j)) __builtin_amdgcn_s_setprio(3);
  MmaItem T;
  if (!mma_find(desc, count, pc, b, j, blockIdx.x * (blockDim.x >> 6) + w, T)) return;
  if (!T.I.active) return;
  v16i D[7];
  mma_accum(D, T, 0, 1, Wm, lds);
  mma_apply(D, T.I, T.cc, T.c, T.r, T.active, T.q2, rd, (int)(threadIdx.x & 63));
}

// The near launches on the matrix cores (the in-panel columns and the next
// panel's: few columns, on the critical path): one workgroup per item, its
// four wavefronts splitting the panel columns k between them (k0 + w, k0 +
// w + 4, ...), their int32 products summed by LDS atomic adds (exact, so
// the order does not matter), and wavefront 0 applying the result.  The
// waves take the SIMDs' issue slots ahead of the bulk launch's.  LDS: four
// C byte planes per wavefront, then the 7 x 16 x 64 int32 sums.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_update_mma_sk(const InstDesc* __restrict__ desc, int count, int pc, int b,
                                                     int j, int rd, int Wm) {
  extern __shared__ int64_t smem[];
  __builtin_amdgcn_s_setprio(3);
  const int lane = threadIdx.x & 63, w = uni(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int PB = mma_plane_bytes(Wm);
  uint32_t* lds = (uint32_t*)smem + w * PB;
  int32_t* sum = (int32_t*)((uint32_t*)smem + nw * PB);
  MmaItem T;
  if (!mma_find(desc, count, pc, b, j, blockIdx.x, T)) return;   // uniform over the workgroup
  if (!T.I.active) return;
  for (int x = threadIdx.x; x < 7 * 16 * 64; x += blockDim.x) sum[x] = 0;
  __syncthreads();
  v16i D[7];
  mma_accum(D, T, w, nw, Wm, lds);
#pragma unroll
  for (int s = 0; s < 7; s++)
#pragma unroll
    for (int v = 0; v < 16; v++) __hip_atomic_fetch_add(sum + (s * 16 + v) * 64 + lane, D[s][v], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int s = 0; s < 7; s++)
#pragma unroll
    for (int v = 0; v < 16; v++) D[s][v] = sum[(s * 16 + v) * 64 + lane];
  mma_apply(D, T.I, T.cc, T.c, T.r, T.active, T.q2, rd, lane);
}

struct FinOut {
  int nbal;       // balanced digits of the result (top nonzero + 1)
  int nstd;       // standard digits of |result|
  int neg;        // sign of the result
  int bits;       // bit length of |result|
  uint32_t topv;  // top standard digit
};

// LDS ordering among the lanes of the one wavefront that runs a
// wave_resolve / wave_finalize: a workgroup barrier when that wavefront is the
// whole workgroup (BLK), else a wavefront-scope fence and wave barrier, so
// that other wavefronts of a larger workgroup need not take part.
template <bool BLK>
__device__ __forceinline__ void lds_sync() {
  if constexpr (BLK) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Carry resolution over nblk blocks of 16 digits held in LDS (x), one
// wavefront: block q absorbs the carry cin[q] coming from block q-1 and
// renormalises (balanced or standard digits), handing its own carry to block
// q+1 in the next round; rounds repeat until no carry is left inside the
// number (at most nblk rounds).  cin[0] may hold a carry into block 0.
// Returns the total carry out of the top block.
template <bool BAL, bool BLK = true, int FB = WB>
__device__ int64_t wave_resolve(int32_t* x, int nblk, int64_t* cin, int64_t* cout) {
  const int lane = threadIdx.x & 63;
  int64_t top = cin[nblk];   // carry already out of the top block
  for (int round = 0; round <= nblk + 1; round++) {
    int any = 0;
    for (int q = lane; q < nblk; q += 64) {
      const int64_t c = cin[q];
      int64_t v = c;
      if (c != 0) {
        for (int m = 0; m < FB; m++) {
          v += x[q * FB + m];
          const int32_t d = BAL ? balanced29(v) : (int32_t)(v & (RADIX - 1));
          x[q * FB + m] = d;
          v = (v - d) >> DB;
        }
      }
      cout[q + 1] = v;
      any |= (v != 0) && (q + 1 < nblk);
    }
    lds_sync<BLK>();
    top += cout[nblk];
    if (!__any(any)) break;
    for (int q = lane; q < nblk; q += 64) cin[q] = q == 0 ? 0 : cout[q];
    lds_sync<BLK>();
  }
  lds_sync<BLK>();
  return top;
}

// RNE(value / 2^h) of one lazily represented number by one wavefront: the
// value (lazy digits Ap[s as], W a multiple of 16, pending block carries
// Kp[q ks] for q >= 1) is normalised block by block in parallel,
// its sign taken from the top digit, its magnitude converted to standard
// digits, shifted right by h bits with round-to-nearest-even, and written as
// balanced digits (Cr) and standard magnitude digits (Sr), cap each.  Each
// lane normalises blocks of FB digits (a divisor of 16) one digit after
// another; the carries between blocks are then resolved in rounds.  LDS:
// dg and ob of W + 48 int32, ca and cb of W/FB + 8 int64.
template <bool BLK = true, int FB = WB, bool PRE = false, typename CT, typename ST>
__device__ FinOut wave_finalize(const int32_t* Ap, int64_t as, int W, const int64_t* Kp, int64_t ks,
                                int h, CT Cr, ST Sr, int cap, GLOBAL int32_t* flags,
                                int32_t* dg, int32_t* ob, int64_t* ca, int64_t* cb,
                                const int64_t* Psub = nullptr, uint32_t* Sl = nullptr) {
  const int lane = threadIdx.x & 63;
  const int nb = W / FB;
  // 1. load, block-local balanced normalisation, carries between blocks (the
  // pending carries Kp belong to the 16-digit blocks of the update).  PRE:
  // the caller has already put the digits in dg and the carries in cb.
  for (int q = lane; q < nb; q += 64) {
    int32_t a[FB];
    const int q16 = q * FB / WB;
    int64_t v = 0;
    if constexpr (PRE) {
#pragma unroll
      for (int m = 0; m < FB; m++) a[m] = dg[q * FB + m];
      if (q16 > 0 && q * FB == q16 * WB) v = cb[q16];
    } else {
#pragma unroll
      for (int m = 0; m < FB; m++) a[m] = Ap[(int64_t)(q * FB + m) * as];
      if (q16 > 0 && q * FB == q16 * WB) v = Kp[(int64_t)q16 * ks];
    }
#pragma unroll
    for (int m = 0; m < FB; m++) {
      v += a[m];
      if (Psub) v -= Psub[q * FB + m];
      const int32_t d = balanced29(v);
      dg[q * FB + m] = d;
      v = (v - d) >> DB;
    }
    ca[q + 1] = v;
  }
  if (lane == 0) ca[0] = 0;
  lds_sync<BLK>();
  // carries out of block q were stored in ca[q+1]: the carry into block q
  if (wave_resolve<true, BLK, FB>(dg, nb, ca, cb) != 0 && lane == 0) gor(flags, 2);
  // 2. sign: the top nonzero digit
  int mytop = -1;
  for (int s = lane; s < W; s += 64) if (dg[s] != 0) mytop = s;
  const int top = wave_max(mytop);
  const bool neg = top >= 0 && dg[top] < 0;
  lds_sync<BLK>();
  // 3. magnitude as standard digits
  for (int q = lane; q < nb; q += 64) {
    int64_t v = 0;
#pragma unroll
    for (int m = 0; m < FB; m++) {
      const int64_t x = (int64_t)(neg ? -dg[q * FB + m] : dg[q * FB + m]) + v;
      const int32_t u = (int32_t)(x & (RADIX - 1));
      dg[q * FB + m] = u;
      v = x >> DB;
    }
    ca[q + 1] = v;
  }
  if (lane == 0) ca[0] = 0;
  lds_sync<BLK>();
  wave_resolve<false, BLK, FB>(dg, nb, ca, cb);
  // 4. shift right by h bits; round to nearest, ties to even
  const int hq = h / DB, hb = h % DB;
  const int hbit_digit = (h - 1) / DB, hbit = (h - 1) % DB;
  const int nout = W - hq + 1;                 // output digits incl. a carry digit
  const int nbo = (nout + FB - 1) / FB;
  for (int i = lane; i < nbo * FB; i += 64) {
    uint32_t o = 0;
    if (i < nout) {
      const int s = hq + i;
      const uint32_t lo = s < W ? (uint32_t)dg[s] : 0u;
      const uint32_t hi = s + 1 < W ? (uint32_t)dg[s + 1] : 0u;
      o = (lo >> hb) | (hb ? ((hi << (DB - hb)) & (uint32_t)(RADIX - 1)) : 0u);
    }
    ob[i] = (int32_t)o;
  }
  int st = 0;
  for (int s = lane; s < hbit_digit; s += 64) st |= dg[s] != 0;
  const uint32_t hd = (uint32_t)dg[hbit_digit];
  const int sticky = __any(st) || (hbit > 0 && (hd & ((1u << hbit) - 1)));
  const int half = (hd >> hbit) & 1;
  lds_sync<BLK>();
  const int inc = half && (sticky || (ob[0] & 1));
  for (int q = lane; q <= nbo; q += 64) ca[q] = (q == 0) ? inc : 0;
  lds_sync<BLK>();
  if (wave_resolve<false, BLK, FB>(ob, nbo, ca, cb) != 0 && lane == 0) gor(flags, 16);
  // 5. standard digits out; balanced copy with the sign
  int ts = -1;
  for (int i = lane; i < nbo * FB; i += 64) {
    const int32_t u = i < nout ? ob[i] : 0;
    if (i < cap) {
      Sr[i] = (uint32_t)u;
      if (Sl) Sl[i] = (uint32_t)u;
    }
    if (u != 0) { ts = i; if (i >= cap) gor(flags, 16); }
  }
  for (int i = nbo * FB + lane; i < cap; i += 64) {
    Sr[i] = 0;
    if (Sl) Sl[i] = 0;
  }
  const int stop = wave_max(ts);
  const uint32_t topv = stop >= 0 ? (uint32_t)ob[stop] : 0u;
  lds_sync<BLK>();
  for (int q = lane; q < nbo; q += 64) {
    int64_t v = 0;
#pragma unroll
    for (int m = 0; m < FB; m++) {
      v += ob[q * FB + m];
      const int32_t d = balanced29(v);
      ob[q * FB + m] = d;
      v = (v - d) >> DB;
    }
    ca[q + 1] = v;
  }
  if (lane == 0) ca[0] = 0;
  lds_sync<BLK>();
  const int64_t extra = wave_resolve<true, BLK, FB>(ob, nbo, ca, cb);   // 0 or 1: one more digit
  int tb = -1;
  for (int i = lane; i < cap; i += 64) {
    int32_t d = i < nbo * FB ? ob[i] : 0;
    if (i == nbo * FB) d = (int32_t)extra;
    d = neg ? -d : d;
    Cr[i] = d;
    if (d != 0) tb = i;
  }
  if (extra != 0 && nbo * FB >= cap && lane == 0) gor(flags, 16);
  FinOut f;
  f.nbal = wave_max(tb) + 1;
  f.nstd = stop + 1;
  f.neg = neg ? 1 : 0;
  f.bits = stop < 0 ? 0 : DB * stop + (32 - __clz(topv));
  f.topv = topv;
  return f;
}

// Carries between the register blocks of one number: lane l holds digits
// [R l, R l + R) (l < nbl), already normalised within its block; c is
// the carry entering the block.  Each round every block absorbs its carry
// (balanced or standard digits) and hands its own to the lane above by a DPP
// wave shift, until no carry crosses a boundary below the top block.
// Returns the total carry out of the top block.
template <bool BAL, int R>
__device__ __forceinline__ int64_t reg_resolve(int64_t* d, int64_t c, int nbl) {
  const int lane = threadIdx.x & 63;
  int64_t top = 0;
  for (int round = 0; round <= 64; round++) {
    if (!__any(c != 0)) break;
    int64_t v = c;
    if (c != 0) {
      v = 0;
      int64_t t = c;
#pragma unroll
      for (int m = 0; m < R; m++) {
        t += d[m];
        const int64_t nd = BAL ? (int64_t)balanced29(t) : (t & (RADIX - 1));
        d[m] = nd;
        t = (t - nd) >> DB;
      }
      v = t;
    }
    top += lane_read(v, nbl - 1);
    c = lane_shr1(lane < nbl - 1 ? v : 0);
  }
  return top;
}

// wave_finalize with the number in registers (W and the W - h/29 + 1 output
// digits at most 64 R): the same
// steps (block normalisation, sign, magnitude, shift by h with RNE, standard
// and balanced outputs) and the same results and flags, but every carry
// moves between lanes by DPP shifts instead of LDS rounds.  Inputs as in
// wave_finalize's PRE form (lazy digits in dg, pending 16-block carries in
// cb, optional subtrahend Psub); ob (W + 48 int32) is scratch for the shift.
template <bool BLK, int R, typename CT, typename ST>
__device__ __forceinline__ FinOut wave_finalize_reg(int W, int h, CT Cr, ST Sr, int cap, GLOBAL int32_t* flags,
                                    const int32_t* dg, int32_t* ob, const int64_t* cb,
                                    const int64_t* Psub, uint32_t* Sl) {
  const int lane = threadIdx.x & 63;
  const int nbl = W / R;
  const bool own = lane < nbl;
  int64_t d[R];
  // 1. load, block normalisation to balanced digits, carries between blocks
  {
    const int s0 = R * lane;
    const int sl = own ? s0 : 0;
    int64_t kv = cb[sl / WB];
    int32_t gv[R];
    int64_t pv[R];
#pragma unroll
    for (int m = 0; m < R; m++) gv[m] = dg[sl + m];
    if (Psub) {
#pragma unroll
      for (int m = 0; m < R; m++) pv[m] = Psub[sl + m];
    } else {
#pragma unroll
      for (int m = 0; m < R; m++) pv[m] = 0;
    }
    pin(kv);
#pragma unroll
    for (int m = 0; m < R; m++) {
      pin(gv[m]);
      pin(pv[m]);
    }
    int64_t t = own && s0 >= WB && s0 % WB == 0 ? kv : 0;
#pragma unroll
    for (int m = 0; m < R; m++) {
      const int64_t x = own ? (int64_t)gv[m] - pv[m] : 0;
      t += x;
      d[m] = balanced29(t);
      t = (t - d[m]) >> DB;
    }
    const int64_t top = lane_read(t, nbl - 1) + reg_resolve<true, R>(d, lane_shr1(lane < nbl - 1 ? t : 0), nbl);
    if (top != 0 && lane == 0) gor(flags, 2);
  }
  // 2. sign: the top nonzero digit
  int mytop = -1, mysign = 0;
#pragma unroll
  for (int m = 0; m < R; m++)
    if (own && d[m] != 0) {
      mytop = R * lane + m;
      mysign = d[m] < 0;
    }
  const int top = wave_max_mono(mytop);
  const bool neg = top >= 0 && __builtin_amdgcn_readlane(mysign, top / R) != 0;
  // 3. magnitude as standard digits
  {
    int64_t t = 0;
#pragma unroll
    for (int m = 0; m < R; m++) {
      t += neg ? -d[m] : d[m];
      d[m] = t & (RADIX - 1);
      t >>= DB;
    }
    (void)reg_resolve<false, R>(d, lane_shr1(lane < nbl - 1 ? t : 0), nbl);
  }
  // 4. shift right by h bits through LDS; round to nearest, ties to even
  uint32_t* ls = (uint32_t*)ob;
#pragma unroll
  for (int m = 0; m < R; m++) if (own) ls[R * lane + m] = (uint32_t)d[m];
  for (int x = W + lane; x < W + R + 2; x += 64) ls[x] = 0;
  lds_sync<BLK>();
  const int hq = h / DB, hb = h % DB;
  const int hbit_digit = (h - 1) / DB, hbit = (h - 1) % DB;
  const int nout = W - hq + 1;
  const int nbo = (nout + R - 1) / R;
  int64_t o[R];
  uint32_t lv[R + 1];
#pragma unroll
  for (int m = 0; m <= R; m++) lv[m] = ls[min(hq + R * lane + m, W - 1)];
#pragma unroll
  for (int m = 0; m <= R; m++) pin(lv[m]);
#pragma unroll
  for (int m = 0; m < R; m++) {
    const int i = R * lane + m;
    const int s2 = hq + i;
    const uint32_t lo = s2 < W ? lv[m] : 0u;
    const uint32_t hi = s2 + 1 < W ? lv[m + 1] : 0u;
    const uint32_t v = (lo >> hb) | (hb ? ((hi << (DB - hb)) & (uint32_t)(RADIX - 1)) : 0u);
    o[m] = i < nout ? v : 0u;
  }
  int st = 0;
#pragma unroll
  for (int m = 0; m < R; m++) if (own && R * lane + m < hbit_digit && d[m] != 0) st = 1;
  const uint32_t hd = ls[hbit_digit];
  const int sticky = __any(st) || (hbit > 0 && (hd & ((1u << hbit) - 1)));
  const int half = (hd >> hbit) & 1;
  const int inc = half && (sticky || (lane_read(o[0], 0) & 1));
  if (reg_resolve<false, R>(o, lane == 0 ? inc : 0, nbo) != 0 && lane == 0) gor(flags, 16);
  // 5. standard digits out; balanced copy with the sign
  int ts = -1;
  uint32_t tv = 0;
#pragma unroll
  for (int m = 0; m < R; m++) {
    const int i = R * lane + m;
    if (lane >= nbo) continue;
    const uint32_t u = i < nout ? (uint32_t)o[m] : 0u;
    if (i < cap) {
      Sr[i] = u;
      if (Sl) Sl[i] = u;
    }
    if (u != 0) {
      ts = i;
      tv = u;
      if (i >= cap) gor(flags, 16);
    }
  }
  for (int i = nbo * R + lane; i < cap; i += 64) {
    Sr[i] = 0;
    if (Sl) Sl[i] = 0;
  }
  const int stop = wave_max_mono(ts);
  const uint32_t topv = stop >= 0 ? (uint32_t)__builtin_amdgcn_readlane((int32_t)tv, stop / R) : 0u;
  {
    int64_t t = 0;
#pragma unroll
    for (int m = 0; m < R; m++) {
      t += lane < nbo ? o[m] : 0;
      o[m] = balanced29(t);
      t = (t - o[m]) >> DB;
    }
    const int64_t extra = lane_read(t, nbo - 1) + reg_resolve<true, R>(o, lane_shr1(lane < nbo - 1 ? t : 0), nbo);
    int tb = -1;
#pragma unroll
    for (int m = 0; m < R; m++) {
      const int i = R * lane + m;
      if (lane >= nbo) continue;
      const int32_t v = (int32_t)(neg ? -o[m] : o[m]);
      if (i < cap) {
        Cr[i] = v;
        if (v != 0) tb = i;
      } else if (v != 0) {
        gor(flags, 16);
      }
    }
    for (int i = nbo * R + lane; i < cap; i += 64) Cr[i] = i == nbo * R ? (int32_t)(neg ? -extra : extra) : 0;
    if (extra != 0 && nbo * R >= cap && lane == 0) gor(flags, 16);
    FinOut f;
    // the extra digit, when it is there and fits, is the top one
    f.nbal = extra != 0 && nbo * R < cap ? nbo * R + 1 : wave_max_mono(tb) + 1;
    f.nstd = stop + 1;
    f.neg = neg ? 1 : 0;
    f.bits = stop < 0 ? 0 : DB * stop + (32 - __clz(topv));
    f.topv = topv;
    return f;
  }
}

// Quotient digits taken per pass over the remainder and zero positions kept
// below position 0.  divide_entry's DNIR is the number of 64-position groups
// of divisor digits its bulk pass holds in registers (larger divisors read
// the rest from LDS).
constexpr int DQ = 8;
static_assert(DQ == 8, "bulk_sum pairs the DQ products as s and s + 4");
constexpr int DOFF = DQ + 4;

// The bulk subtraction of divide_entry at remainder position b + rel:
// x - sum_s q[s] dd[rel + s + 1 - DQ], the DQ products summed in four
// independent chains (the empty asm statements keep the compiler from
// folding them back into one dependent chain of multiply-adds).
__device__ __forceinline__ int64_t bulk_sum(int64_t x, const int32_t* q, const int32_t* ddv) {
  int64_t a[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    a[k] = (int64_t)(-q[k]) * (int64_t)ddv[k];
    a[k] += (int64_t)(-q[k + 4]) * (int64_t)ddv[k + 4];
    asm volatile("" : "+v"(a[k]));
  }
  return x + ((a[0] + a[1]) + (a[2] + a[3]));
}

// Carry-save split of one 64-position group of bulk sums: the digit in
// [0, 2^29) plus the carry of the position below, moved one lane up by a DPP
// wave shift whose vacated lane 0 is filled, by a DPP wave rotation, with the
// top lane of the previous group's carries (prev; zero for the first group),
// so no carry passes through a scalar register.  Returns the new remainder
// value of this lane's position; prev becomes this group's carries.
__device__ __forceinline__ int64_t bulk_split(int64_t x, int64_t& prev) {
  const int64_t lo = x & (RADIX - 1);
  const int64_t hi = x >> DB;
  const int32_t f0 = __builtin_amdgcn_update_dpp(0, (int32_t)prev, 0x13C, 0xf, 0xf, false);
  const int32_t f1 = __builtin_amdgcn_update_dpp(0, (int32_t)(prev >> 32), 0x13C, 0xf, 0xf, false);
  const int32_t h0 = __builtin_amdgcn_update_dpp(f0, (int32_t)hi, 0x138, 0xf, 0xf, false);
  const int32_t h1 = __builtin_amdgcn_update_dpp(f1, (int32_t)(hi >> 32), 0x138, 0xf, 0xf, false);
  prev = hi;
  return lo + (int64_t)(((uint64_t)(uint32_t)h1 << 32) | (uint32_t)h0);
}

// The bulk pass over the first G 64-position groups, whose divisor digits sit
// in registers (DDL): all loads first, then the sums, then the splits in
// order with the carries passing upward.
template <int G>
__device__ __forceinline__ void bulk_groups(int64_t* rem, int b, int nbulk, const int32_t* q,
                                            int32_t (*DDL)[DQ], int top_group, int64_t& prev,
                                            int64_t& htop) {
  const int lane = threadIdx.x & 63;
  int64_t xv[G];
#pragma unroll
  for (int i = 0; i < G; i++) xv[i] = rem[b + min(lane + 64 * i, max(nbulk - 1, 0))];
#pragma unroll
  for (int i = 0; i < G; i++) pin(xv[i]);
#pragma unroll
  for (int i = 0; i < G; i++) xv[i] = bulk_sum(lane + 64 * i < nbulk ? xv[i] : 0, q, DDL[i]);
#pragma unroll
  for (int i = 0; i < G; i++) {
    const int rel = lane + 64 * i;
    const int64_t v = bulk_split(xv[i], prev);
    if (rel < nbulk) rem[b + rel] = v;
    if (i == top_group) htop = prev;
  }
}

// Destination of the byte planes of one L entry (row of ColInfo::l8off):
// byte s of digit j at p[s ps + (j / 32) cs + j % 32], digits [0, n) written
// (zeros above the quotient); p == nullptr when there are none.
struct L8Out {
  GLOBAL int8_t* p;
  int64_t ps, cs;
  int n;
};
__device__ __forceinline__ void l8_store(const L8Out& o, int j, int32_t d) {
  int32_t b0, b1, b2, b3;
  split_bytes(d, b0, b1, b2, b3);
  GLOBAL int8_t* q = o.p + (int64_t)(j >> 5) * o.cs + (j & 31);
  q[0] = (int8_t)b0;
  q[o.ps] = (int8_t)b1;
  q[2 * o.ps] = (int8_t)b2;
  q[3 * o.ps] = (int8_t)b3;
}
__device__ __forceinline__ void l8_zero(const L8Out& o, int from) {
  if (!o.p) return;
  for (int j = from + (int)(threadIdx.x & 63); j < o.n; j += 64) l8_store(o, j, 0);
}

// out = RNE(+-|num| 2^h / |d|) for one 64-lane workgroup: schoolbook long
// division in radix 2^29 with a lazily normalised int64 remainder in LDS.
// num: standard digits Sr[0..ns) of its magnitude, sign negN; divisor:
// standard digits Dp[0..nd) of |d| 2^sh (top digit >= 2^28), sign negd.  Each
// quotient digit is estimated from the top three remainder digits against the
// top three divisor digits in float64 (error < 1/2 + 2^-20), so quotient
// digits are signed and the remainder stays within (1/2 + eps) |d|; the final
// remainder decides the rounding (ties to even).  The top DQ + 4 remainder
// positions live in registers of every lane (identical in all lanes), where
// DQ quotient digits are found one after another; then one pass over the
// positions below subtracts all DQ multiples of the divisor at once, one
// position per lane, with carry-save normalisation.  Writes `cap` balanced
// digits to out[j * os] (zero filled) and returns the digit count.
template <bool BLK = true, int DNIR = 4>
__device__ __forceinline__ int divide_entry(int64_t* smem, const uint32_t* Sr, int ns, int negN,
                            const uint32_t* Dp, int nd, int sh, int negd, int h, GLOBAL int32_t* out,
                            int64_t os, int cap, GLOBAL int32_t* out2, int64_t os2, GLOBAL int32_t* flags,
                            L8Out o8 = L8Out{nullptr, 0, 0, 0}) {
  const int lane = threadIdx.x & 63;
  nd = __builtin_amdgcn_readfirstlane(nd);
  ns = __builtin_amdgcn_readfirstlane(ns);
  if (nd == 0) {
    for (int j = lane; j < cap; j += 64) { out[(int64_t)j * os] = 0; if (out2) out2[(int64_t)j * os2] = 0; }
    l8_zero(o8, 0);
    if (lane == 0) gor(flags, 4);
    return 0;
  }
  const int Sbits = h + sh, Sq = Sbits / DB, Sb = Sbits % DB;
  const int nu = ns == 0 ? 0 : Sq + ns + 1;
  if (nu < nd) {  // quotient below 2 / 2^29: rounds to zero
    for (int j = lane; j < cap; j += 64) { out[(int64_t)j * os] = 0; if (out2) out2[(int64_t)j * os2] = 0; }
    l8_zero(o8, 0);
    return 0;
  }
  int64_t* rem = smem + DOFF;                // positions -DOFF .. nu + 2
  // the divisor digits with zeros around them: DPAD below, up to the
  // register groups' reach above, so that every register of the divisor
  // below is one unconditional LDS read
  static_assert(DNIR >= 1 && DNIR <= 8, "divide_shm sizes the divisor padding for at most 8 groups");
  constexpr int DPAD = 16, DHI = 64 * DNIR + 16;
  int64_t* dd = rem + (nu + 3) + DPAD;       // dd[-DPAD .. nd + DHI)
  int64_t* qd = dd + nd + DHI;               // nu - nd + 2
  // (the loads of a fill are issued unconditionally from clamped indices and
  // pinned by an empty asm statement, so the compiler cannot sink each one
  // into a branch of its own with a wait behind it)
  for (int i = lane; i < nd; i += 64) dd[i] = (int64_t)Dp[i];
  for (int i = lane - DPAD; i < 0; i += 64) dd[i] = 0;
  for (int i = nd + lane; i < nd + DHI; i += 64) dd[i] = 0;
  for (int s = lane - DOFF; s < Sq; s += 64) rem[s] = 0;
  for (int s = nu + lane; s < nu + 3; s += 64) rem[s] = 0;
  for (int s = Sq + lane; s < nu; s += 64) {
    const int i = s - Sq;                    // 0 .. ns
    uint32_t a = Sr[min(i, ns - 1)], b = Sr[max(i - 1, 0)];
    asm volatile("" : "+v"(a), "+v"(b));
    const uint64_t av = i < ns ? a : 0u, bv = i >= 1 ? b : 0u;
    rem[s] = (int64_t)(((av << Sb) | (Sb ? (bv >> (DB - Sb)) : 0)) & (RADIX - 1));
  }
  const int jmax = __builtin_amdgcn_readfirstlane(nu - nd);
  for (int j = lane; j <= jmax + 1; j += 64) qd[j] = 0;
  lds_sync<BLK>();
  const double R = (double)RADIX;
  const double D3 = (double)dd[nd - 1] * R * R + (double)dd[nd - 2] * R + (double)dd[nd - 3];
  const double ninvD = -R / D3;   // (negated) quotient estimates by one multiply
  // top divisor digits for the register window: DT[m] = dd[nd - 1 - m]
  int32_t DT[DQ + 2];
#pragma unroll
  for (int m = 0; m < DQ + 2; m++) DT[m] = (int32_t)dd[nd - 1 - m];
  // bulk positions of a pass: b + rel, rel = lane + 64 i in [0, nd - 3); the
  // divisor digit that q[s] meets there is dd[rel + s + 1 - DQ], the same in
  // every pass (zero beyond the divisor, so groups past the last are inert)
  const int nbulk = nd - 3;
  const int NI = nbulk > 0 ? (nbulk + 63) / 64 : 0;
  const int top_group = __builtin_amdgcn_readfirstlane(nbulk > 0 ? (nbulk - 1) / 64 : -1);
  const int top_lane = __builtin_amdgcn_readfirstlane(nbulk > 0 ? (nbulk - 1) & 63 : 0);
  int32_t DDL[DNIR][DQ];
#pragma unroll
  for (int i = 0; i < DNIR; i++)
#pragma unroll
    for (int s = 0; s < DQ; s++) DDL[i][s] = (int32_t)dd[lane + 64 * i + s + 1 - DQ];
  // register window: W[x] holds remainder position T + 1 - x
  int T = __builtin_amdgcn_readfirstlane(nu);
  int64_t W[DQ + 4];
#pragma unroll
  for (int x = 0; x < DQ + 4; x++) W[x] = rem[T + 1 - x];
  int j0 = jmax;
  while (true) {
    const int Qe = min(DQ, j0 + 1);
    int32_t q[DQ];
#pragma unroll
    for (int s = 0; s < DQ; s++) {
      q[s] = 0;
      if (s < Qe) {
        // quotient digit j0 - s: fold position t + 1 into t, carry t - 1
        // upward, estimate from t, t - 1 and the lazy t - 2 (|W| < 2^63 there:
        // converting it to double costs at most 2^10 of its units)
        W[s + 1] += W[s] << DB;
        W[s] = 0;
        const int64_t cy = W[s + 2] >> DB;
        W[s + 2] &= RADIX - 1;
        W[s + 1] += cy;
        // |W[s+1]| < 2^31 here
        const double Tv = fma((double)(int32_t)W[s + 1], R * R, fma((double)(int32_t)W[s + 2], R, (double)W[s + 3]));
        // -q, with |q| < 2^30 and divisor digits < 2^29: one 32 x 32 -> 64
        // multiply-add each
        const int32_t nq = (int32_t)rint(Tv * ninvD);
        q[s] = -nq;
#pragma unroll
        for (int x = s + 2; x < DQ + 4; x++) W[x] += (int64_t)nq * (int64_t)DT[x - s - 2];
      }
    }
    {  // quotient digits j0 .. j0 - Qe + 1 to LDS, one lane each
      int32_t v = q[0];
#pragma unroll
      for (int s = 1; s < DQ; s++) v = lane == s ? q[s] : v;
      if (lane < Qe) qd[j0 - lane] = v;
    }
    // every position below the window: subtract the DQ multiples at once.
    // The register groups (only the first when the divisor needs no more)
    // load and sum independently, then split in order, the carries passing
    // upward; groups beyond them take their divisor digits from LDS.
    const int b = j0 - DQ + 1;
    int64_t prev = 0, htop = 0;
    // (as many register groups as the divisor has, in steps of powers of two)
    if (NI <= 1) bulk_groups<1>(rem, b, nbulk, q, DDL, top_group, prev, htop);
    else if (DNIR > 2 && NI <= 2) bulk_groups<(DNIR > 2 ? 2 : DNIR)>(rem, b, nbulk, q, DDL, top_group, prev, htop);
    else if (DNIR > 4 && NI <= 4) bulk_groups<(DNIR > 4 ? 4 : DNIR)>(rem, b, nbulk, q, DDL, top_group, prev, htop);
    else bulk_groups<DNIR>(rem, b, nbulk, q, DDL, top_group, prev, htop);
    for (int i = DNIR; i < NI; i++) {
      // (dd[nd] is zero, so the divisor digit index clamps to nd)
      int32_t ddv[DQ];
#pragma unroll
      for (int s = 0; s < DQ; s++) ddv[s] = (int32_t)dd[min(lane + 64 * i + s + 1 - DQ, nd)];
      const int rel = lane + 64 * i;
      int64_t xr = rem[b + min(rel, max(nbulk - 1, 0))];
      pin(xr);
#pragma unroll
      for (int s = 0; s < DQ; s++) pin(ddv[s]);
      const int64_t x = bulk_sum(rel < nbulk ? xr : 0, q, ddv);
      const int64_t v = bulk_split(x, prev);
      if (rel < nbulk) rem[b + rel] = v;
      if (i == top_group) htop = prev;
    }
    // the top bulk position's carry enters the window's lowest position
    if (top_group >= 0) W[DQ + 3] += lane_read(htop, top_lane);
    lds_sync<BLK>();
    if (j0 - DQ < 0) break;
    T -= DQ;
    j0 -= DQ;
#pragma unroll
    for (int x = 0; x < 4; x++) W[x] = W[x + DQ];
#pragma unroll
    for (int x = 4; x < DQ + 4; x++) W[x] = rem[T + 1 - x];
  }
  // final remainder: its top positions nd + 1 .. nd - 2 are the window
  // entries j0 .. j0 + 3 (T = nd + j0 after the last pass), folded and
  // carried in registers by every lane alike; the rounding decision follows
  // from remainder / divisor in float64 unless that is within 1e-6 of a tie,
  // when the whole remainder goes back to LDS for an exact comparison
  int64_t r1 = 0, r0 = 0, rm1 = 0, rm2 = 0;
#pragma unroll
  for (int x = 0; x < DQ + 4; x++) {
    r1 = x == j0 ? W[x] : r1;
    r0 = x == j0 + 1 ? W[x] : r0;
    rm1 = x == j0 + 2 ? W[x] : rm1;
    rm2 = x == j0 + 3 ? W[x] : rm2;
  }
  r0 += r1 << DB;
  if (nd >= 2) {
    const int64_t cy = rm2 >> DB;
    rm2 -= cy << DB;
    rm1 += cy;
  }
  {
    const int64_t cy = rm1 >> DB;
    rm1 -= cy << DB;
    r0 += cy;
  }
  const double Tr = (double)r0 * R * R + (double)rm1 * R + (nd >= 2 ? (double)rm2 : 0.0);
  const double f = Tr * R / D3;   // remainder / divisor
  const double af = fabs(f);
  int adj = af > 0.5 ? (f > 0 ? 1 : -1) : 0;
  if (uni(fabs(2.0 * af - 1.0) <= 1e-6)) {
    if (lane == 0) {
#pragma unroll
      for (int x = 0; x < DQ + 4; x++) rem[T + 1 - x] = W[x];
      rem[nd + 1] = 0;
      rem[nd] = r0;
      rem[nd - 1] = rm1;
      if (nd >= 2) rem[nd - 2] = rm2;
    }
    lds_sync<BLK>();
    if (lane == 0) {
      // exact comparison of 2 rem with +d and -d
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
      adj = 0;
      if (s1 > 0) adj = 1;
      else if (s1 == 0) adj = odd ? 1 : 0;
      else if (s2 < 0) adj = -1;
      else if (s2 == 0) adj = odd ? -1 : 0;
    }
    adj = uni(adj);
  }
  // quotient digits -> balanced digits (one carry step suffices: |q| <= 2^30)
  const int nq = jmax + 2;
  int mytop = -1;
  const int sgn = (negN ^ negd) ? -1 : 1;
  const int nqc = min(nq, cap);
  for (int j = lane; j < nqc; j += 64) {
    // (the rounding adjustment belongs to digit 0)
    int64_t x = qd[j], y = qd[max(j - 1, 0)];
    pin(x);
    pin(y);
    x += j == 0 ? adj : 0;
    y += j == 1 ? adj : 0;
    int64_t o = balanced29(x);
    if (j >= 1) o += (y - balanced29(y)) >> DB;
    const int32_t od = (int32_t)(sgn * o);
    out[(int64_t)j * os] = od;
    if (out2) out2[(int64_t)j * os2] = od;
    if (o8.p) l8_store(o8, j, od);
    if (od != 0) mytop = j;
  }
  for (int j = nqc + lane; j < cap; j += 64) {
    out[(int64_t)j * os] = 0;
    if (out2) out2[(int64_t)j * os2] = 0;
  }
  l8_zero(o8, nqc);
  if (nq > cap && lane == 0) {
    for (int j = cap; j < nq; j++) {
      const int64_t x = (j <= jmax ? qd[j] : 0) + (j == 0 ? adj : 0);
      int64_t o = balanced29(x);
      if (j - 1 <= jmax) {
        const int64_t y = qd[j - 1] + (j == 1 ? adj : 0);
        o += (y - balanced29(y)) >> DB;
      }
      if (o != 0) gor(flags, 8);
    }
  }
  return wave_max_strided(mytop, (cap - 1) >> 6) + 1;
}

// Digits per lane-serial block in the column finalisations (short serial
// chains, more lanes busy).
constexpr int FIN_FB = 4;

// The finalisation of the column and solve kernels (digits already in dg,
// carries in cb): in registers, 2 or 8 digits a lane, while the number and
// the shifted result both fit 64 lanes, else through LDS.
template <typename CT, typename ST>
__device__ __forceinline__ FinOut finalize_pre(int W, int h, CT Cr, ST Sr, int cap, GLOBAL int32_t* flags,
                                               int32_t* dg, int32_t* ob, int64_t* ca, int64_t* cb,
                                               const int64_t* Psub, uint32_t* Sl = nullptr) {
  const int nout = W - h / DB + 1;
  if (W <= 64 * 2 && nout <= 64 * 2)
    return wave_finalize_reg<false, 2>(W, h, Cr, Sr, cap, flags, dg, ob, cb, Psub, Sl);
  if (W <= 64 * 8 && nout <= 64 * 8)
    return wave_finalize_reg<false, 8>(W, h, Cr, Sr, cap, flags, dg, ob, cb, Psub, Sl);
  if (W <= 64 * 16 && nout <= 64 * 16)
    return wave_finalize_reg<false, 16>(W, h, Cr, Sr, cap, flags, dg, ob, cb, Psub, Sl);
  return wave_finalize<false, FIN_FB, true>(nullptr, 0, W, nullptr, 0, h, Cr, Sr, cap, flags, dg, ob, ca, cb,
                                            Psub, Sl);
}


// |d| 2^sh as standard digits, top digit in [2^28, 2^29): every output digit
// takes its own input digit shifted up and the top bits of the one below
template <typename SP, typename OP>
__device__ __forceinline__ void normalise_divisor(SP S, int n, int sh, OP out) {
  for (int i = threadIdx.x & 63; i < n; i += 64) {
    const uint32_t lo = i > 0 && sh > 0 ? S[i - 1] >> (DB - sh) : 0u;
    out[i] = ((S[i] << sh) | lo) & (uint32_t)(RADIX - 1);
  }
}


template <int PB>
__device__ __forceinline__ void renorm_pb(int64_t* acc) {
#pragma unroll
  for (int m = 0; m < PB; m++) {
    const int64_t hc = acc[m] >> DB;
    acc[m] -= hc << DB;
    acc[m + 1] += hc;
  }
}

// P[0..W) = the digits of the exact product Lr * Cp by one wavefront, lazily
// normalised (|P[s]| < 2^36).  Lr: nL balanced digits in LDS, zero padded to
// a multiple of 8; Cp: nC balanced digits in LDS.  Lane l forms the output
// digits [PB l, PB l + PB) of each pass of 64 PB by operand scanning over Lr
// (PB a power of two up to 8),
// with the PB digits of C it meets held in a ring of registers (one new digit
// per step), then adds its carry into the digit above in a second phase.
// PB = 2 covers W <= 128 in one pass with every lane busy; PB = 8 suits wide
// entries.  A product wider than W digits sets bit 1 of flags[0], like an
// update that overflows its entry.
template <int PB, bool BLK>
__device__ __forceinline__ void near_product(const int32_t* Lr, int nL, const int32_t* Cp, int nC, int W, int64_t* P,
                             int32_t* flags) {
  const int lane = threadIdx.x & 63;
  if (lane == 0 && nL > 0 && nC > 0 && nL + nC - 1 > W) atomicOr(&flags[0], 1);
  for (int s = lane; s < W; s += 64) P[s] = 0;
  lds_sync<BLK>();
  if (nL <= 0 || nC <= 0) return;
  const int nL8 = (nL + 7) / 8 * 8;
  for (int p0 = 0; p0 < W; p0 += 64 * PB) {
    const int s0 = p0 + PB * lane;
    int64_t acc[PB + 1];
    int32_t ring[PB];   // ring[(s0 + b - a) mod PB] = C[s0 + b - a]
#pragma unroll
    for (int m = 0; m <= PB; m++) acc[m] = 0;
#pragma unroll
    for (int b = 0; b < PB; b++) ring[b] = s0 + b < nC ? Cp[s0 + b] : 0;
    int cnt = 0;
    for (int a0 = 0; a0 < nL8; a0 += 8) {
      // eight steps: their L digits and the C digits entering the ring are
      // read up front so the LDS reads overlap
      // (C digits from clamped indices, pinned together by an empty asm
      // statement and masked afterwards: no branch and wait per read)
      int32_t la[8], cn[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        la[u] = Lr[a0 + u];
        cn[u] = Cp[min(max(s0 - (a0 + u) - 1, 0), nC - 1)];
      }
      asm volatile("" : "+v"(cn[0]), "+v"(cn[1]), "+v"(cn[2]), "+v"(cn[3]), "+v"(cn[4]), "+v"(cn[5]),
                   "+v"(cn[6]), "+v"(cn[7]));
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int idx = s0 - (a0 + u) - 1;
        cn[u] = idx >= 0 && idx < nC ? cn[u] : 0;
      }
#pragma unroll
      for (int u = 0; u < 8; u++) {
#pragma unroll
        for (int b = 0; b < PB; b++) acc[b] += (int64_t)la[u] * (int64_t)ring[(b - u) & (PB - 1)];
        ring[(PB - 1 - u) & (PB - 1)] = cn[u];
      }
      cnt += 8;
      if (cnt >= 96) { renorm_pb<PB>(acc); cnt = 0; }
    }
    renorm_pb<PB>(acc);
#pragma unroll
    for (int b = 0; b < PB; b++)
      if (s0 + b < W) P[s0 + b] += acc[b];
    lds_sync<BLK>();
    if (s0 + PB < W) P[s0 + PB] += acc[PB];
    else if (s0 < W && acc[PB] != 0) atomicOr(&flags[0], 1);
    lds_sync<BLK>();
  }
}

// LDS of the pivot's balanced and standard digits while it is finalised
__host__ __device__ inline int pivot_scratch_bytes(int CW) { return 8 * CW; }

// One column c in one launch: C = RNE(A / 2^h) for every row r in [c, N) and
// L = RNE(C 2^h / d) for r > c.  Workgroups [0, n_near) are the rows: one
// 128-lane workgroup per (instance, row); wavefront 0 finalises row r while
// wavefront 1 finalises the pivot row c into LDS (the workgroup of row c
// writes the pivot out, with its normalised divisor digits and the inertia
// flags), then wavefront 0 divides row r by the pivot.  With upd (the
// in-kernel look-ahead schedule, rank-1 updates), both first subtract the
// update of their entry by column c - 1 (L_{c-1}[r] C_{c-1}[c], formed in
// LDS) while normalising, and the remaining workgroups apply the update by
// column c - 1 to the columns [c + 1, N), two items each; the next launch
// finds every column it needs complete.  The accumulator, its carries
// (plane rd) and the update's operands are read into LDS in one batch of
// loads.  LDS: the pivot's normalised divisor, this row's standard digits and
// the pivot's shift and sign (piv_bytes, live to the end), then either the
// pivot's balanced and standard digits with the two product + finalisation
// regions (fin_bytes each), or, once those are dead, the division.
template <int DNIR>
__device__ __forceinline__ void column_step(const InstDesc* __restrict__ desc, int count, int c, int n_near,
                                            int rd, int upd, int fin_bytes, int piv_bytes) {
  if ((int)blockIdx.x >= n_near) {
    if (upd && c > 0)
      update_item(desc, count, c - 1, 1, UPD_FAR, (c - 1) & 1,
                  ((int)blockIdx.x - n_near) * 2 + uni(threadIdx.x >> 6));
    return;
  }
  extern __shared__ int64_t smem[];
  // the row chain is the launch's critical path: its waves take the SIMDs'
  // issue slots ahead of update waves that share them
  __builtin_amdgcn_s_setprio(3);
  int bid = blockIdx.x, inst = -1;
  for (int i = 0; i < count; i++) {
    const int n = max(0, gp(desc)[i].N - c);
    if (bid < n) { inst = i; break; }
    bid -= n;
  }
  if (inst < 0) return;
  const InstDesc I = desc[inst];
  if (!I.active) return;
  const int N = I.N;
  const int r = c + bid, lr = r - c;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const ColInfo cc = I.cols[c];
  const int W = cc.W;
  // this row's L^T placement, used only by the division at the end: loaded
  // now so that its latency hides behind the row's first phases
  const int64_t cr_ltoff = gp(I.cols)[r].ltoff;
  const int cr_PT = gp(I.cols)[r].PT;
  char* base = (char*)smem;
  uint32_t* pD = (uint32_t*)base;            // pivot's normalised divisor
  uint32_t* oS = pD + cc.CW;                 // this row's standard digits
  int* pinfo = (int*)(oS + cc.CW);           // pivot: standard digits, shift, sign
  int32_t* pC = (int32_t*)(base + piv_bytes);
  uint32_t* pS = (uint32_t*)(pC + cc.CW);
  char* wbase = base + piv_bytes + pivot_scratch_bytes(cc.CW) + wave * fin_bytes;
  int32_t* dg = (int32_t*)wbase;
  int32_t* ob = dg + (W + 48);
  int64_t* ca = (int64_t*)(ob + (W + 48));
  int64_t* cb = ca + (W / FIN_FB + 8);
  int64_t* Pd = cb + (W / FIN_FB + 8);           // product digits, W
  int64_t* dsm = (int64_t*)(base + piv_bytes);
  const GLOBAL int64_t* Kc = gp(I.Kc + cc.koff + (int64_t)rd * cc.nb * cc.R);
  GLOBAL uint32_t* Srow = gp(I.S + cc.soff + (int64_t)lr * cc.CW);
  const GLOBAL int32_t* Ag = gp(I.A + cc.aoff);
  GLOBAL int32_t* flg = gp(I.flags);
  // the row this wavefront finalises
  const int fr = wave == 0 ? r : c;
  const bool work = wave == 0 || r != c;
  const int64_t* Psub = nullptr;
  // the accumulator digits and pending carries of entry (fr, c), and the
  // operands of its update by column c - 1 (digits up to their capacities,
  // which are zero filled), all requested before the first store to LDS so
  // that their latencies overlap
  const int flr = fr - c;
  const bool updr = upd && work && c > 0;
  const ColInfo ck = I.cols[c > 0 ? c - 1 : 0];
  const GLOBAL int32_t* Lsrc = gp(I.L + ck.loff + (fr - (c - 1)));
  const GLOBAL int32_t* Csrc = gp(I.C + ck.coff + (int64_t)ck.CW);
  int32_t* Lr = (int32_t*)(Pd + W);            // L_{c-1}[fr], LW + 8
  int32_t* Cp = Lr + (ck.LW + 8);              // C_{c-1}[c], CW
  constexpr int U = 8;
  int32_t av[U], lv[U], cv[U];
  int64_t kv = 0;
  int nL = 0, nC = 0;
  if (work) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int x = lane + 64 * u;
      av[u] = x < W ? Ag[(int64_t)x * cc.R + flr] : 0;
      lv[u] = updr && x < ck.LW ? Lsrc[(int64_t)x * ck.R] : 0;
      cv[u] = updr && x < ck.CW ? Csrc[x] : 0;
    }
    kv = lane > 0 && lane < cc.nb ? Kc[(int64_t)lane * cc.R + flr] : 0;
    if (updr) {
      nL = min(gp(I.nL)[tri_index(N, c - 1, fr)], ck.LW);
      nC = min(gp(I.nC)[tri_index(N, c - 1, c)], ck.CW);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int x = lane + 64 * u;
      if (x < W) dg[x] = av[u];
      if (updr && x < ck.LW) Lr[x] = lv[u];
      if (updr && x < ck.CW) Cp[x] = cv[u];
    }
    if (lane < cc.nb) cb[lane] = kv;
    for (int x = lane + 64 * U; x < W; x += 64) dg[x] = Ag[(int64_t)x * cc.R + flr];
    for (int q = lane + 64; q < cc.nb; q += 64) cb[q] = Kc[(int64_t)q * cc.R + flr];
    if (updr) {
      for (int x = lane + 64 * U; x < ck.LW; x += 64) Lr[x] = Lsrc[(int64_t)x * ck.R];
      for (int x = lane + 64 * U; x < ck.CW; x += 64) Cp[x] = Csrc[x];
      for (int x = ck.LW + lane; x < ck.LW + 8; x += 64) Lr[x] = 0;
    }
  }
  if (updr) {
    lds_sync<false>();
    if (W <= 128) near_product<2, false>(Lr, nL, Cp, nC, W, Pd, I.flags);
    else near_product<8, false>(Lr, nL, Cp, nC, W, Pd, I.flags);
    Psub = Pd;
  }
  if (work) lds_sync<false>();
  FinOut f;
  f.nstd = 0;
  f.neg = 0;
  if (wave == 0) {
    f = finalize_pre(W, I.h, gp(I.C + cc.coff + (int64_t)lr * cc.CW), Srow, cc.CW, flg, dg, ob, ca, cb, Psub,
                     oS);
    const int64_t ti = tri_index(N, c, r);
    if (lane == 0) {
      gp(I.nC)[ti] = f.nbal;
      gp(I.nCs)[ti] = f.neg ? -f.nstd : f.nstd;
      gp(I.b32C)[ti] = (f.bits + 31) / 32;
    }
    if (r == c) {
      const int sh = f.nstd > 0 ? 28 - (31 - __clz(f.topv)) : 0;
      if (lane == 0) {
        if (f.nstd == 0 || f.neg) {
          __hip_atomic_fetch_min(flg + 1, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (f.nstd > 0 && f.neg) __hip_atomic_fetch_add(flg + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        GLOBAL int32_t* di = gp(I.dinfo);
        di[4 * c] = f.nstd;
        di[4 * c + 1] = sh;
        di[4 * c + 2] = f.nstd > 0 ? f.neg : 0;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      normalise_divisor(Srow, f.nstd, sh, gp(I.D + cc.doff));
    }
  } else if (work) {
    const FinOut p = finalize_pre(W, I.h, pC, pS, cc.CW, flg, dg, ob, ca, cb, Psub);
    const int sh = p.nstd > 0 ? 28 - (31 - __clz(p.topv)) : 0;
    lds_sync<false>();
    normalise_divisor(pS, p.nstd, sh, pD);
    if (lane == 0) {
      pinfo[0] = p.nstd;
      pinfo[1] = sh;
      pinfo[2] = p.nstd > 0 ? p.neg : 0;
    }
  }
  __syncthreads();
  if (r == c || wave != 0) return;
  const L8Out o8{gp(I.L8 + cc.l8off + (int64_t)lr * 32), (int64_t)cc.G * cc.R * 32, (int64_t)cc.R * 32, 32 * cc.G};
  const int n = divide_entry<false, DNIR>(dsm, oS, f.nstd, f.neg, pD, pinfo[0], pinfo[1], pinfo[2], I.h,
                                    gp(I.L + cc.loff + lr), cc.R, cc.LW, gp(I.LT + cr_ltoff + c), cr_PT, flg, o8);
  if (lane == 0) {
    gp(I.nL)[tri_index(N, c, r)] = n;
    if (n > cc.LW - 2 * WB) gor(flg, 8);
  }
}

// The in-kernel look-ahead schedule: three waves per SIMD (at most 168
// registers, two divisor groups in registers) keep the update workgroups of
// the launch from starving for occupancy.
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3)))
k_column(const InstDesc* __restrict__ desc, int count, int c, int n_near, int fin_bytes, int piv_bytes) {
  column_step<2>(desc, count, c, n_near, (c + 1) & 1, 1, fin_bytes, piv_bytes);
}

// Finalisation and division alone (the update came from k_update launches).
__global__ void __launch_bounds__(128) k_fdiv(const InstDesc* __restrict__ desc, int count, int c, int rd,
                                              int n_near, int fin_bytes, int piv_bytes) {
  column_step<8>(desc, count, c, n_near, rd, 0, fin_bytes, piv_bytes);
}

// v_i = RNE(y_i 2^K / m) with the common divisor m (standard digits of m 2^sh
// in md[0..nd)); y_i as standard magnitude digits (us rows, signed nUs)
__global__ void __launch_bounds__(64) k_vscale(int K, const uint32_t* __restrict__ us,
                                               const int32_t* __restrict__ nUs, int VW,
                                               const uint32_t* __restrict__ md, int nd, int sh,
                                               int32_t* __restrict__ out, int32_t* __restrict__ flags) {
  extern __shared__ int64_t smem[];
  const int i = blockIdx.x;
  const int nsg = nUs[i];
  divide_entry(smem, us + (int64_t)i * VW, nsg < 0 ? -nsg : nsg, nsg < 0, md, nd, sh, 0, K,
               gp(out + (int64_t)i * VW), 1, VW, nullptr, 0, gp(flags));
}

// ---------------------------------------------------------------- solves
// Accumulators of a vector: VA digit planes of Npad rows (value of row i =
// sum_s acc[s Npad + i] 2^(29 s) plus pending block carries), the same lazy
// format and double-buffered carries as the matrix columns.


// acc_i -= sum_{k0 <= k < k1} V_k[i] u_k for rows i in [i_lo, i_hi):
//   forward (bwd = 0): V_k[i] = L_k[i] (column layout), rows i > k;
//   backward (bwd = 1): V_k[i] = L_i[k] (row layout L^T), rows i < k.
// u_k (uniform): row k of ub (VW balanced digits, nU[k] used).  Work item
// `it` of T * nbA (T row tiles of 64, nbA digit blocks) for one wavefront.
__device__ __forceinline__ void vupdate_item(const ColInfo* __restrict__ cols, int N, int bwd, int k0,
                                             int k1, int i_lo, int i_hi, int rd, int it,
                                             int32_t* __restrict__ acc, int64_t* __restrict__ kc,
                                             int Npad, int nbA, const int32_t* __restrict__ ub,
                                             const int32_t* __restrict__ nU, int VW,
                                             const int32_t* __restrict__ Lb,
                                             const int32_t* __restrict__ LTb,
                                             const int32_t* __restrict__ nLw, int LWT,
                                             int32_t* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int T = (i_hi - i_lo + 63) / 64;
  const int q = uni(it / T);
  const int t = uni(it - q * T);
  const int i = i_lo + 64 * t + lane;
  const bool active = i < i_hi;
  const int ii = active ? i : i_hi - 1;
  int64_t a[WB + 1];
#pragma unroll
  for (int m = 0; m <= WB; m++) a[m] = 0;
  int cnt = 0;
  for (int k = k0; k < k1; k++) {
    const int nC = min(uni(nU[k]), VW - WB);
    int nLl, lo, cap, P;
    const int32_t* Lp;
    int64_t nbytes;
    const ColInfo kk = cols[k];
    if (!bwd) {
      nLl = active ? nLw[tri_index(N, k, ii)] : 0;
      Lp = Lb + kk.loff;
      nbytes = (int64_t)kk.LW * kk.R * 4;
      lo = ii - k;
      P = kk.R;
      cap = kk.LW;
    } else {
      nLl = active ? nLw[tri_index(N, ii, k)] : 0;
      Lp = LTb + kk.ltoff;
      nbytes = (int64_t)LWT * kk.PT * 4;
      lo = ii;
      P = kk.PT;
      cap = cols[ii].LW;
    }
    const int nL = min(uni(wave_max(min(nLl, cap - 2 * WB))), LWT - 2 * WB);
    accum_block(a, cnt, ub + (int64_t)k * VW, nC, Lp, nbytes, lo, P, nL, q);
  }
  if (!active) return;
  apply_block(a, uptr(acc), (int64_t)nbA * WB * Npad * 4, i, Npad, q,
              q > 0 ? gp(kc + ((int64_t)rd * nbA + q) * Npad + i) : nullptr,
              q + 1 < nbA ? gp(kc + ((int64_t)(rd ^ 1) * nbA + q + 1) * Npad + i) : nullptr, gp(flags));
}




// ---------------------------------------------- batched inverse iteration
// One SweepArgs per instance; blockIdx.y (or blockIdx.x for one-workgroup
// kernels) selects the instance.

__global__ void __launch_bounds__(256) k_vinit_b(const SweepArgs* __restrict__ args, int stage) {
  const SweepArgs& a = args[blockIdx.y];
  const int32_t* src = stage == 0 ? a.v : a.wb;
  const int Sbits = stage == 0 ? a.h + a.gbits : a.h;
  const int Sq = Sbits / DB, Sb = Sbits % DB;
  const int64_t n = (int64_t)a.VA * a.Npad;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(idx / a.Npad), i = (int)(idx - (int64_t)s * a.Npad);
    int64_t v = 0;
    if (i < a.N) {
      const int j = s - Sq;
      if (j >= 0 && j < a.VW) v += (((int64_t)src[(int64_t)i * a.VW + j]) << Sb) & (RADIX - 1);
      if (j - 1 >= 0 && j - 1 < a.VW) v += (((int64_t)src[(int64_t)i * a.VW + j - 1]) << Sb) >> DB;
    }
    a.acc[idx] = (int32_t)v;
  }
  const int64_t nk = (int64_t)2 * a.nbA * a.Npad;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nk;
       idx += (int64_t)gridDim.x * blockDim.x)
    a.kc[idx] = 0;
}

__global__ void __launch_bounds__(64) k_vdivide_b(const SweepArgs* __restrict__ args) {
  extern __shared__ int64_t smem[];
  const SweepArgs& a = args[blockIdx.y];
  const int k = blockIdx.x;
  if (k >= a.N) return;
  const int nsg = a.nUs[k];
  divide_entry(smem, a.us + (int64_t)k * a.VW, nsg < 0 ? -nsg : nsg, nsg < 0, a.Dd + a.cols[k].doff,
                   a.dinfo[4 * k], a.dinfo[4 * k + 1], a.dinfo[4 * k + 2], a.h, gp(a.wb + (int64_t)k * a.VW), 1,
                   a.VW, nullptr, 0, gp(a.flags));
}


// One column step of a substitution sweep for every instance (blockIdx.y),
// with the previous column's update folded in, so a sweep is one launch per
// column.  Forward (bwd = 0): column k, previous column p = k - 1; backward
// (bwd = 1): column k, p = k + 1 (rows below are done first).  The first
// wavefront of workgroup 0 subtracts the product V_p[k] u_p from acc_k while
// normalising it (V = L, or L^T backward; the accumulator, its carries and
// the operands read into LDS in one batch) and finalises u_k; every other
// wavefront is an update item (vupdate_item) applying column p to the rows beyond k
// (forward [k + 1, N), backward [0, k)).  Carry planes: the update at step j
// reads plane (j - 1) & 1 and writes j & 1, so row k finds its carries in
// plane (j + 1) & 1.  LDS (workgroup 0): finalisation, product digits, V and
// u rows.
__global__ void __launch_bounds__(256) k_vcol_b(const SweepArgs* __restrict__ args, int bwd, int k, int j,
                                                int fin_bytes) {
  extern __shared__ int64_t smem[];
  const SweepArgs& a = args[blockIdx.y];
  const int N = a.N;
  if (k >= N) return;
  const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int p = bwd ? k + 1 : k - 1;
  const bool has_p = p >= 0 && p < N;
  if (blockIdx.x > 0 || wave > 0) {
    if (!has_p) return;
    const int it = (int)blockIdx.x * 4 + wave - 1;
    const int i_lo = bwd ? 0 : k + 1, i_hi = bwd ? k : N;
    if (i_hi <= i_lo) return;
    const int T = (i_hi - i_lo + 63) / 64;
    if (it >= T * a.nbA) return;
    vupdate_item(a.cols, N, bwd, p, p + 1, i_lo, i_hi, (j - 1) & 1, it, a.acc, a.kc, a.Npad, a.nbA, a.ub, a.nU,
                 a.VW, a.L, a.LT, a.nL, a.LWT, a.flags);
    return;
  }
  __builtin_amdgcn_s_setprio(3);   // the sweep's critical path (see column_step)
  const int VA = a.VA;
  int32_t* dg = (int32_t*)smem;
  int32_t* ob = dg + (VA + 48);
  int64_t* ca = (int64_t*)(ob + (VA + 48));
  int64_t* cb = ca + (VA / FIN_FB + 8);
  int64_t* Pd = cb + (VA / FIN_FB + 8);        // product digits, VA
  const int rd = (j + 1) & 1;
  const GLOBAL int64_t* Kc = gp(a.kc + (int64_t)rd * a.nbA * a.Npad + k);
  const GLOBAL int32_t* accg = gp(a.acc + k);
  const GLOBAL int32_t* ubg = gp(a.ub);
  // the operands of the row's update by column p: V digits (stride P) and u_p
  const ColInfo cp = a.cols[has_p ? p : k];
  const GLOBAL int32_t* Vsrc = gp(bwd ? a.LT + cp.ltoff + k : a.L + cp.loff + 1);
  const int Vstride = bwd ? cp.PT : cp.R;
  const int Vcap = bwd ? min(a.cols[k].LW, a.LWT) : cp.LW;
  int32_t* Lr = (int32_t*)(Pd + VA);           // Vcap + 8
  int32_t* Up = Lr + (Vcap + 8);               // VW
  constexpr int U = 4;
  int32_t av[U], lv[U], uv[U];
  int64_t kv = 0;
  int nL = 0, nC = 0;
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int x = lane + 64 * u;
    av[u] = x < VA ? accg[(int64_t)x * a.Npad] : 0;
    lv[u] = has_p && x < Vcap ? Vsrc[(int64_t)x * Vstride] : 0;
    uv[u] = has_p && x < a.VW ? ubg[(int64_t)p * a.VW + x] : 0;
  }
  kv = lane > 0 && lane < a.nbA ? Kc[(int64_t)lane * a.Npad] : 0;
  if (has_p) {
    nL = min(gp(a.nL)[bwd ? tri_index(N, k, p) : tri_index(N, p, k)], Vcap - 2 * WB);
    nL = min(nL, a.LWT - 2 * WB);
    nC = min(gp(a.nU)[p], a.VW - WB);
  }
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int x = lane + 64 * u;
    if (x < VA) dg[x] = av[u];
    if (has_p && x < Vcap) Lr[x] = lv[u];
    if (has_p && x < a.VW) Up[x] = uv[u];
  }
  if (lane < a.nbA) cb[lane] = kv;
  for (int x = lane + 64 * U; x < VA; x += 64) dg[x] = accg[(int64_t)x * a.Npad];
  for (int q = lane + 64; q < a.nbA; q += 64) cb[q] = Kc[(int64_t)q * a.Npad];
  const int64_t* Psub = nullptr;
  if (has_p) {
    for (int x = lane + 64 * U; x < Vcap; x += 64) Lr[x] = Vsrc[(int64_t)x * Vstride];
    for (int x = lane + 64 * U; x < a.VW; x += 64) Up[x] = ubg[(int64_t)p * a.VW + x];
    for (int x = Vcap + lane; x < Vcap + 8; x += 64) Lr[x] = 0;
    lds_sync<false>();
    if (VA <= 128) near_product<2, false>(Lr, nL, Up, nC, VA, Pd, a.flags);
    else near_product<8, false>(Lr, nL, Up, nC, VA, Pd, a.flags);
    Psub = Pd;
  }
  lds_sync<false>();
  const FinOut f = finalize_pre(VA, a.h, gp(a.ub + (int64_t)k * a.VW), gp(a.us + (int64_t)k * a.VW), a.VW,
                                gp(a.flags), dg, ob, ca, cb, Psub);
  if (lane == 0) {
    gp(a.nU)[k] = f.nbal;
    gp(a.nUs)[k] = f.neg ? -f.nstd : f.nstd;
    if (f.nbal > a.VW - WB) gor(gp(a.flags), 32);
  }
  // the backward sweep's result; each lane copies the digits it wrote itself
  if (bwd && a.y)
    for (int x = lane; x < a.VW; x += 64) gp(a.y)[(int64_t)k * a.VW + x] = gp(a.ub)[(int64_t)k * a.VW + x];
}


// <v, y> (which = 0) and <v, v> (which = 1) exactly, split over DOT_PARTS
// workgroups per dot (each a subset of the rows; the host adds the parts):
// thread t owns output digit positions p = t, t + 256, ... and sums
// v_i[a] y_i[p - a] over its rows i
// and digits a in int64, moving everything above 29 bits into a second
// accumulator every 64 products.  Rows are staged in LDS (v_i broadcast,
// y_i read at consecutive addresses).  Written as two lazy int64 digit rows,
// dots[which][0][p] (low parts, position p) and dots[which][1][p] (high
// parts of position p - 1): value = sum over both rows of d_p 2^(29 p).
// LDS: 2 VW int32.
__global__ void __launch_bounds__(256) k_vdots_b(const SweepArgs* __restrict__ args) {
  extern __shared__ int64_t smem[];
  const SweepArgs& a = args[blockIdx.x];
  const int which = blockIdx.y;       // 0: <v, y>, 1: <v, v>
  const int part = blockIdx.z;        // rows i = part, part + DOT_PARTS, ...
  const int32_t* V = a.v;
  const int32_t* Y = which == 0 ? a.y : a.v;
  const int VW = a.VW, np = VW + 4;     // 2 np = 2 VW + 8 entries per row
  int64_t* lo_row = a.dots + ((int64_t)which * DOT_PARTS + part) * 2 * (2 * np);
  int64_t* hi_row = lo_row + 2 * np;
  int32_t* vs = (int32_t*)smem;
  int32_t* ys = vs + VW;
  constexpr int PT = 4;                  // output positions per thread and pass
  for (int p = threadIdx.x; p < 2 * np; p += blockDim.x) {
    if (p >= 2 * VW) lo_row[p] = 0;
    if (p == 0 || p > 2 * VW) hi_row[p] = 0;
  }
  for (int base = 0; base < 2 * VW; base += PT * 256) {
    int64_t lo[PT], hi[PT];
    int cnt[PT];
#pragma unroll
    for (int u = 0; u < PT; u++) { lo[u] = 0; hi[u] = 0; cnt[u] = 0; }
    for (int i = part; i < a.N; i += DOT_PARTS) {
      __syncthreads();
      for (int d = threadIdx.x; d < VW; d += blockDim.x) {
        vs[d] = V[(int64_t)i * VW + d];
        ys[d] = Y[(int64_t)i * VW + d];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < PT; u++) {
        const int p = base + threadIdx.x + 256 * u;
        if (p < 2 * VW) {
          const int a_lo = max(0, p - VW + 1), a_hi = min(p, VW - 1);
          for (int d = a_lo; d <= a_hi; d++) {
            lo[u] += (int64_t)vs[d] * (int64_t)ys[p - d];
            if (++cnt[u] == 64) {
              cnt[u] = 0;
              hi[u] += lo[u] >> DB;
              lo[u] &= RADIX - 1;
            }
          }
        }
      }
    }
    // lo belongs to position p, hi to position p + 1
#pragma unroll
    for (int u = 0; u < PT; u++) {
      const int p = base + threadIdx.x + 256 * u;
      if (p < 2 * VW) {
        lo_row[p] = lo[u];
        hi_row[p + 1] = hi[u];
      }
    }
  }
}

// the row of largest |y| (standard magnitude digits us, signed counts nUs):
// per lane the best of its rows, then a tournament over the wavefront;
// its magnitude shifted so that the top digit has bit 28 set goes to md, and
// mdinfo = {digits, shift, row}
__device__ __forceinline__ int cmp_mag_rows(const uint32_t* us, const int32_t* nUs, int VW, int i, int j) {
  const int ni = abs(nUs[i]), nj = abs(nUs[j]);
  if (ni != nj) return ni > nj ? 1 : -1;
  for (int d = ni - 1; d >= 0; d--) {
    const uint32_t x = us[(int64_t)i * VW + d], y = us[(int64_t)j * VW + d];
    if (x != y) return x > y ? 1 : -1;
  }
  return 0;
}

__global__ void __launch_bounds__(64) k_vmax_b(const SweepArgs* __restrict__ args) {
  const SweepArgs& a = args[blockIdx.x];
  const int lane = threadIdx.x;
  int best = -1;
  for (int i = lane; i < a.N; i += 64)
    if (best < 0 || cmp_mag_rows(a.us, a.nUs, a.VW, i, best) > 0) best = i;
  for (int o = 1; o < 64; o <<= 1) {
    const int other = __shfl_xor(best, o, 64);
    if (other >= 0 && (best < 0 || cmp_mag_rows(a.us, a.nUs, a.VW, other, best) > 0 ||
                       (cmp_mag_rows(a.us, a.nUs, a.VW, other, best) == 0 && other < best)))
      best = other;
  }
  if (lane != 0) return;
  const int nstd = best >= 0 ? abs(a.nUs[best]) : 0;
  if (nstd == 0) {
    a.mdinfo[0] = 0; a.mdinfo[1] = 0; a.mdinfo[2] = best;
    return;
  }
  const uint32_t* row = a.us + (int64_t)best * a.VW;
  const int sh = 28 - (31 - __clz(row[nstd - 1]));
  uint32_t carry = 0;
  for (int d = 0; d < nstd; d++) {
    const uint64_t x = ((uint64_t)row[d] << sh) | carry;
    a.md[d] = (uint32_t)(x & (RADIX - 1));
    carry = (uint32_t)(x >> DB);
  }
  a.mdinfo[0] = nstd;
  a.mdinfo[1] = sh;
  a.mdinfo[2] = best;
}

__global__ void __launch_bounds__(64) k_vscale_b(const SweepArgs* __restrict__ args) {
  extern __shared__ int64_t smem[];
  const SweepArgs& a = args[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= a.N) return;
  const int nsg = a.nUs[i];
  divide_entry(smem, a.us + (int64_t)i * a.VW, nsg < 0 ? -nsg : nsg, nsg < 0, a.md, a.mdinfo[0],
                   a.mdinfo[1], 0, a.K, gp(a.v + (int64_t)i * a.VW), 1, a.VW, nullptr, 0, gp(a.flags));
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

// pivots d_k = C_k[k] of every instance gathered into rows of ld digits
// (instance i at rows [i maxN, i maxN + N_i))
__global__ void k_gather_pivots(const InstDesc* __restrict__ desc, int maxN, int ld,
                                int32_t* __restrict__ out) {
  const InstDesc I = desc[blockIdx.y];
  const int k = blockIdx.x;
  if (k >= I.N) return;
  const ColInfo kk = I.cols[k];
  int32_t* o = out + ((int64_t)blockIdx.y * maxN + k) * ld;
  for (int i = threadIdx.x; i < ld; i += blockDim.x) o[i] = i < kk.CW ? I.C[kk.coff + i] : 0;
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
hipError_t launch_expand(const BatchView& B, hipStream_t s) {
  hipLaunchKernelGGL(k_expand, dim3(B.maxN, (unsigned)B.plans.size()), dim3(256), 0, s, B.ddesc);
  return hipGetLastError();
}
int64_t update_items(const Plan& P, int pc, int b, int j) {
  int k0, k1, c_lo, c_hi;
  if (!update_range(P.N, pc, b, j, k0, k1, c_lo, c_hi)) return 0;
  return (int64_t)P.itemStart[c_hi] - P.itemStart[c_lo];
}
// With t0 and t1 (timing-capable events, both or neither) the launch's own
// start and end are recorded on them (the dispatch packet's timestamps, as a
// profiler sees the kernel), or, when nothing is launched, the current point
// on both.
static hipError_t mark_empty(hipEvent_t t0, hipEvent_t t1, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (t0) e = hipEventRecord(t0, s);
  if (e == hipSuccess && t1) e = hipEventRecord(t1, s);
  return e;
}
// The widest column of a batch when its updates run on the matrix cores,
// else 0: off when HK_MMA=0, when the int32 accumulators could overflow (b
// panel columns of up to Wm digits: b Wm must stay below 2^15), or when the
// near launches' LDS would exceed the device's.
int mma_width(const BatchView& B, int b) {
  static const int off = [] {
    const char* v = getenv("HK_MMA");
    return v && v[0] == '0' && v[1] == 0;
  }();
  if (off || !B.mma) return 0;
  int Wm = 0;
  for (const Plan* p : B.plans) Wm = std::max(Wm, p->maxW);
  if ((int64_t)std::max(b, 1) * Wm >= 32768 - 64) return 0;
  // the near launches' LDS: four waves' C planes and the int32 sums
  if ((size_t)16 * mma_plane_bytes(Wm) + 7 * 16 * 64 * sizeof(int32_t) > device_lds_limit()) return 0;
  return Wm;
}

hipError_t launch_update(const BatchView& B, int pc, int b, int j, int rd, hipStream_t s, hipEvent_t t0,
                         hipEvent_t t1) {
  int64_t items = 0;
  for (const Plan* p : B.plans) items += update_items(*p, pc, b, j);
  if (items <= 0) return mark_empty(t0, t1, s);
  const int ipw = B.ipw == 1 || B.ipw == 2 ? B.ipw : 4;
  const dim3 grid((unsigned)((items + ipw - 1) / ipw)), block(64 * ipw);
  const int Wm = mma_width(B, b);
  if (Wm > 0 && (update_is_bulk(j) || j == UPD_NEAR) && mma_lds(Wm, b) <= 65536) {
    int64_t tiles = 0;
    for (const Plan* p : B.plans) {
      int k0, k1, c_lo, c_hi;
      if (update_range(p->N, pc, b, j, k0, k1, c_lo, c_hi))
        for (int t = 0; 32 * t < p->N - c_lo; t++) tiles += mma_tile_count(p->N, c_lo, c_hi, t);
    }
    if (tiles <= 0) return mark_empty(t0, t1, s);
    const int run_len = MMA_RUN;
    const int per = (int)((tiles + 8 * run_len - 1) / (8 * run_len)) * run_len;
    const size_t shm = mma_lds(Wm, b);
    if (t0 || t1)
      hipExtLaunchKernelGGL(k_update_mma, dim3(8u * per), dim3(256), shm, s, t0, t1, 0, B.ddesc,
                            (int)B.plans.size(), pc, b, j, rd, Wm, run_len);
    else
      hipLaunchKernelGGL(k_update_mma, dim3(8u * per), dim3(256), shm, s, B.ddesc, (int)B.plans.size(), pc, b, j,
                         rd, Wm, run_len);
    return hipGetLastError();
  }
  // near launches small enough to leave most of the chip idle split their
  // panel columns over four wavefronts per item; larger ones keep one
  // wavefront per item (the split only adds waves to a launch that fills
  // the chip already)
  if (Wm > 0 && !update_is_bulk(j) && items <= MMA_SPLIT_ITEMS) {
    const size_t shm = (size_t)16 * mma_plane_bytes(Wm) + 7 * 16 * 64 * sizeof(int32_t);
    if (t0 || t1)
      hipExtLaunchKernelGGL(k_update_mma_sk, dim3((unsigned)items), dim3(256), shm, s, t0, t1, 0, B.ddesc,
                            (int)B.plans.size(), pc, b, j, rd, Wm);
    else
      hipLaunchKernelGGL(k_update_mma_sk, dim3((unsigned)items), dim3(256), shm, s, B.ddesc, (int)B.plans.size(), pc,
                         b, j, rd, Wm);
    return hipGetLastError();
  }
  if (Wm > 0) {
    const size_t shm = (size_t)ipw * 4 * mma_plane_bytes(Wm);
    if (t0 || t1)
      hipExtLaunchKernelGGL(k_update_mma_w, grid, block, shm, s, t0, t1, 0, B.ddesc, (int)B.plans.size(), pc, b, j,
                            rd, Wm);
    else
      hipLaunchKernelGGL(k_update_mma_w, grid, block, shm, s, B.ddesc, (int)B.plans.size(), pc, b, j, rd, Wm);
    return hipGetLastError();
  }
  auto kern = update_is_bulk(j) ? k_update : k_update_near;
  if (t0 || t1)
    hipExtLaunchKernelGGL(kern, grid, block, 0, s, t0, t1, 0, B.ddesc, (int)B.plans.size(), pc, b, j, rd);
  else
    hipLaunchKernelGGL(kern, grid, block, 0, s, B.ddesc, (int)B.plans.size(), pc, b, j, rd);
  return hipGetLastError();
}
// LDS of wave_finalize for W digits in blocks of FB
static size_t fin_shm(int W, int FB = WB) {
  return sizeof(int32_t) * 2 * (size_t)(W + 48) + sizeof(int64_t) * 2 * (size_t)(W / FB + 8);
}
// LDS of divide_entry: remainder DOFF + nu + 3, divisor nd with 16 zeros
// below and 64 DNIR + 16 above (DNIR <= 8), quotient nu - nd + 2
static size_t divide_shm(int h, int num_cap, int den_cap) {
  const int Sq = (h + 28) / DB + 1;
  const int nu_max = Sq + num_cap + 1;
  return sizeof(int64_t) * (size_t)((DOFF + nu_max + 3) + (16 + den_cap + 64 * 8 + 16) + (nu_max + 3));
}
// LDS of one row workgroup of the column launches for column c: the live
// pivot region, then the larger of the finalisation phase (pivot scratch and
// two per-wave regions; with the rank-1 look-ahead update, the product digits
// and the update's operands too) and the division.  *fin and *piv receive the
// kernel's fin_bytes and piv_bytes.
static size_t column_lds(const BatchView& B, int c, bool upd, int* fin_out, int* piv_out) {
  size_t fin = 0, piv = 0, pcs = 0, div = 0;
  for (const Plan* p : B.plans)
    if (c < p->N) {
      const ColInfo& cc = p->cols[c];
      size_t f = fin_shm(cc.W, FIN_FB);
      if (upd) {
        const int Lw = c > 0 ? p->cols[c - 1].LW + 8 : 0, Cw = c > 0 ? p->cols[c - 1].CW : 0;
        f += sizeof(int64_t) * (size_t)cc.W + sizeof(int32_t) * (size_t)(Lw + Cw);
      }
      fin = std::max(fin, f);
      piv = std::max(piv, (sizeof(uint32_t) * (2 * (size_t)cc.CW + 4) + 7) / 8 * 8);
      pcs = std::max(pcs, (size_t)pivot_scratch_bytes(cc.CW));
      div = std::max(div, divide_shm(p->h, cc.CW, cc.W + 2));
    }
  fin = (fin + 7) / 8 * 8;
  if (fin_out) *fin_out = (int)fin;
  if (piv_out) *piv_out = (int)piv;
  return piv + std::max(pcs + 2 * fin, div);
}
// LDS of one workgroup of the forward/backward sweep launches
static size_t vcol_lds(const SweepShape& sh) {
  return (fin_shm(sh.maxVA, FIN_FB) + sizeof(int64_t) * (size_t)sh.maxVA +
          sizeof(int32_t) * (size_t)(sh.maxLW + 8 + sh.maxVW) + 7) / 8 * 8;
}
size_t device_lds_limit() {
  static std::mutex mu;
  static int lim[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  std::lock_guard<std::mutex> g(mu);
  if (!lim[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 65536;
    lim[dev] = v;
  }
  return (size_t)lim[dev];
}
std::string factor_lds_check(const BatchView& B, int mode) {
  const size_t lim = device_lds_limit();
  int maxN = 0;
  for (const Plan* p : B.plans) maxN = std::max(maxN, p->N);
  for (int c = 0; c < maxN; c++) {
    const size_t need = column_lds(B, c, mode == 2, nullptr, nullptr);
    if (need > lim)
      return "column " + std::to_string(c) + " needs " + std::to_string(need) +
             " bytes of LDS per workgroup, above the device's " + std::to_string(lim) +
             " (entries too wide: lower N or prec_bits" + (mode == 2 ? ", or use look-ahead mode 0 or 1)" : ")");
  }
  return "";
}
std::string solve_lds_check(const SweepShape& sh) {
  const size_t lim = device_lds_limit();
  const size_t need = std::max(vcol_lds(sh), std::max(sh.shm_div, sh.shm_scale));
  if (need <= lim) return "";
  return "the solve sweeps need " + std::to_string(need) + " bytes of LDS per workgroup, above the device's " +
         std::to_string(lim) + " (vectors too wide: lower N or prec_bits)";
}
hipError_t launch_fdiv(const BatchView& B, int c, int rd, hipStream_t s) {
  int64_t rows = 0;
  for (const Plan* p : B.plans)
    if (c < p->N) rows += p->N - c;
  if (rows <= 0) return hipSuccess;
  int fin = 0, piv = 0;
  const size_t shm = column_lds(B, c, false, &fin, &piv);
  hipLaunchKernelGGL(k_fdiv, dim3((unsigned)rows), dim3(128), shm, s, B.ddesc, (int)B.plans.size(), c, rd,
                     (int)rows, fin, piv);
  return hipGetLastError();
}
hipError_t launch_column(const BatchView& B, int c, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  int64_t rows = 0, items = 0;
  for (const Plan* p : B.plans) {
    if (c < p->N) rows += p->N - c;
    if (c > 0) items += update_items(*p, c - 1, 1, UPD_FAR);
  }
  if (rows <= 0 && items <= 0) return mark_empty(t0, t1, s);
  int fin = 0, piv = 0;
  const size_t shm = column_lds(B, c, true, &fin, &piv);
  const int64_t blocks = rows + (items + 1) / 2;
  if (t0 || t1)
    hipExtLaunchKernelGGL(k_column, dim3((unsigned)blocks), dim3(128), shm, s, t0, t1, 0, B.ddesc,
                          (int)B.plans.size(), c, (int)rows, fin, piv);
  else
    hipLaunchKernelGGL(k_column, dim3((unsigned)blocks), dim3(128), shm, s, B.ddesc, (int)B.plans.size(), c,
                       (int)rows, fin, piv);
  return hipGetLastError();
}
hipError_t launch_gather_pivots_b(const BatchView& B, int32_t* out, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_pivots, dim3(B.maxN, (unsigned)B.plans.size()), dim3(64), 0, s, B.ddesc,
                     B.maxN, ld, out);
  return hipGetLastError();
}
SweepArgs make_sweep_args(const Plan& P, const DevPtrs& D, int panel, int gbits) {
  SweepArgs a;
  memset(&a, 0, sizeof a);
  a.cols = D.cols; a.N = P.N; a.Npad = P.Npad; a.VA = P.VA; a.nbA = P.VA / WB; a.VW = P.VW; a.LWT = P.LWT;
  a.h = P.h; a.bwd = 0; a.panel = panel < 1 ? 1 : panel; a.gbits = gbits; a.K = P.K;
  a.acc = D.acc; a.kc = D.kca; a.ub = D.ub; a.us = D.us; a.nU = D.nU; a.nUs = D.nUs;
  a.L = D.L; a.LT = D.LT; a.nL = D.nL; a.out = nullptr; a.flags = D.flags;
  a.v = D.dv1; a.y = D.dv2; a.wb = D.wb; a.Dd = D.D; a.dinfo = D.dinfo;
  a.dots = D.dots; a.md = D.md; a.mdinfo = D.mdinfo;
  return a;
}
SweepShape sweep_shape(const std::vector<const Plan*>& plans) {
  SweepShape sh;
  sh.count = (int)plans.size();
  for (const Plan* p : plans) {
    sh.maxN = std::max(sh.maxN, p->N);
    sh.maxVA = std::max(sh.maxVA, p->VA);
    sh.maxVW = std::max(sh.maxVW, p->VW);
    sh.maxVAN = std::max(sh.maxVAN, (int64_t)p->VA * p->Npad);
    sh.maxLW = std::max(sh.maxLW, std::max(p->LWT, p->maxW + 32));
    sh.shm_div = std::max(sh.shm_div, divide_shm(p->h, p->VW, p->maxW + 2));
    sh.shm_scale = std::max(sh.shm_scale, divide_shm(p->K, p->VW, p->VW + 2));
  }
  return sh;
}
hipError_t launch_vinit_b(const SweepArgs* args, const SweepShape& sh, int stage, hipStream_t s) {
  const unsigned bx = (unsigned)std::min<int64_t>(blocks_for(sh.maxVAN, 256), 1024);
  hipLaunchKernelGGL(k_vinit_b, dim3(bx, sh.count), dim3(256), 0, s, args, stage);
  return hipGetLastError();
}
hipError_t launch_vcol_b(const SweepArgs* args, const SweepShape& sh, int bwd, int j, hipStream_t s) {
  const int k = bwd ? sh.maxN - 1 - j : j;
  // far rows of the widest instance bound the item count
  const int rows = bwd ? k : sh.maxN - k - 1;
  const int64_t items = j > 0 && rows > 0 ? (int64_t)((rows + 63) / 64) * (sh.maxVA / WB) : 0;
  const size_t fin = vcol_lds(sh);
  hipLaunchKernelGGL(k_vcol_b, dim3((unsigned)((items + 1 + 3) / 4), sh.count), dim3(256), fin, s, args, bwd, k,
                     j, (int)fin);
  return hipGetLastError();
}
hipError_t enqueue_solve(const SweepArgs* args, const SweepShape& sh, hipStream_t s) {
  hipError_t e = launch_vinit_b(args, sh, 0, s);
  for (int j = 0; j < sh.maxN && e == hipSuccess; j++) e = launch_vcol_b(args, sh, 0, j, s);
  if (e == hipSuccess) e = launch_vdivide_b(args, sh, s);
  if (e == hipSuccess) e = launch_vinit_b(args, sh, 1, s);
  for (int j = 0; j < sh.maxN && e == hipSuccess; j++) e = launch_vcol_b(args, sh, 1, j, s);
  return e;
}
hipError_t launch_vdivide_b(const SweepArgs* args, const SweepShape& sh, hipStream_t s) {
  hipLaunchKernelGGL(k_vdivide_b, dim3(sh.maxN, sh.count), dim3(64), sh.shm_div, s, args);
  return hipGetLastError();
}
hipError_t launch_vdots_b(const SweepArgs* args, const SweepShape& sh, hipStream_t s) {
  hipLaunchKernelGGL(k_vdots_b, dim3(sh.count, 2, DOT_PARTS), dim3(256), sizeof(int32_t) * 2 * sh.maxVW, s, args);
  return hipGetLastError();
}
hipError_t launch_vmax_b(const SweepArgs* args, const SweepShape& sh, hipStream_t s) {
  hipLaunchKernelGGL(k_vmax_b, dim3(sh.count), dim3(64), 0, s, args);
  return hipGetLastError();
}
hipError_t launch_vscale_b(const SweepArgs* args, const SweepShape& sh, hipStream_t s) {
  hipLaunchKernelGGL(k_vscale_b, dim3(sh.maxN, sh.count), dim3(64), sh.shm_scale, s, args);
  return hipGetLastError();
}
hipError_t launch_vscale(const Plan& P, const DevPtrs& D, const uint32_t* md, int nd, int sh,
                         int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_vscale, dim3(P.N), dim3(64), divide_shm(P.K, P.VW, nd + 2), s, P.K, D.us, D.nUs, P.VW,
                     md, nd, sh, out, D.flags);
  return hipGetLastError();
}
hipError_t launch_bits(const Plan& P, const DevPtrs& D, hipStream_t s) {
  hipLaunchKernelGGL(k_bitsL, dim3(blocks_for(P.ntri, 256)), dim3(256), 0, s, D.cols, P.N, D.L,
                     D.nL, D.b32L);
  return hipGetLastError();
}

}  // namespace hk
