// Internal declarations shared by the host side and the kernel launchers of
// the hk library.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hk.h"
#include "hk_moments.hpp"
#include "hk_mp.hpp"

struct hk_matrix_s;

namespace hk {

// Device digits: balanced radix 2^29, value = sum_i d_i 2^(29 i) with
// d_i in [-2^28, 2^28) once normalised; stored as int32.
constexpr int DB = 29;
constexpr int64_t RADIX = int64_t(1) << DB;
constexpr int WB = 16;       // digits per output block of the trailing update
constexpr int TROWS = 64;    // rows per update tile (one wavefront)
constexpr int DOT_PARTS = 8; // workgroups per exact dot product (batched inverse iteration)

// Per-column layout record (column c of the working triangle, also used as
// the panel column k that produced C_k / L_k).
struct ColInfo {
  int64_t aoff;   // A: W digit planes of R rows (int32)
  int64_t koff;   // carries: [2][nb][R] (int64)
  int64_t coff;   // C_k rows (N-k) x CW, balanced digits (int32)
  int64_t loff;   // L_k digit planes LW x R (int32), row index r - k
  int64_t soff;   // |C_k| standard digits, rows (N-k) x CW (uint32)
  int64_t doff;   // |d_k| 2^sh standard digits (uint32), W + 2 entries
  int32_t W;      // digits per A entry (multiple of 2 WB)
  int32_t R;      // padded rows (multiple of 64)
  int32_t nb;     // W / WB
  int32_t CW;     // W + 16
  int32_t LW;     // W + 32
  int32_t items;  // trailing-update items of this column: (R/64) * nb
  int64_t ltoff;  // L^T row: entries L_c[r] for c < r, digit planes LWT x PT (int32)
  int32_t PT;     // rows of the L^T planes: r rounded up to 64 (>= 64)
  int32_t G;      // 32-digit chunks of the byte planes of L_k: ceil(LW / 32)
  int64_t l8off;  // byte planes of L_k (int8): [4][G][R][32], digit j of row
                  // r - k at plane s, chunk j / 32, byte j % 32
};

struct Plan {
  int N = 0, K = 0, h = 0;
  uint32_t p = 1, q = 1;
  int WX = 0;                 // digits per moment
  int maxW = 0;
  int gbits = 0;              // solve guard bits
  int VW = 0;                 // digits per vector entry
  int VA = 0;                 // digits per solve accumulator (multiple of WB)
  int Npad = 0;               // N rounded up to 64
  int LWT = 0;                // digit planes of the L^T rows
  std::vector<ColInfo> cols;
  std::vector<int32_t> itemStart;  // N+1 prefix sums of items
  // byte offsets in the workspace
  size_t o_cols, o_items, o_A, o_K, o_C, o_L, o_L8, o_S, o_D, o_dinfo, o_nC, o_nCs, o_nL,
      o_X, o_xs, o_flags, o_b32C, o_b32L, o_vec, o_LT, o_acc, o_kca, o_ub, o_us, o_wb, o_nU,
      o_nUs, o_dv1, o_dv2, o_md, o_mdinfo, o_dots, o_desc, o_sargs, total;
  int64_t ntri;
};

bool make_plan(int N, int64_t bnum, int64_t bden, int K, Plan& P, std::string& err);
int lookahead_mode(int setting, int maxN, int maxW);
// panel width (0: none) and look-ahead (-1: none) from the tuning cache
// named by HK_TUNE_CACHE for this batch shape
struct Schedule { int panel = 0, lookahead = -1, ipw = 0, mma = -1; };
Schedule tuned_schedule(const hk_instance* inst, int count);

// an hk_mpf as an integer with K fractional bits (false if it has more)
bool shift_fixed(const hk_mpf& x, int K, MP& out);

// conversions between host integers and device digits
void mp_to_digits(const MP& v, int32_t* out, int n);          // balanced, zero padded
MP digits_to_mp(const int32_t* d, int n, int64_t stride = 1);

// host threads for the drivers' multiprecision arithmetic: HK_HOST_THREADS
// if set, else the hardware's, at most 16
int host_threads();

// f(i) for every i in [0, n) on up to `threads` host threads, i dealt out
// round-robin (costs that fall or rise with i stay balanced).  A thread the
// system will not start leaves its share to the calling thread.
template <class Fn>
void parallel_for(int n, int threads, Fn&& f) {
  threads = std::max(1, std::min(threads, n));
  if (threads == 1) {
    for (int i = 0; i < n; i++) f(i);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(threads - 1);
  int started = 1;
  for (int t = 1; t < threads; t++, started++) {
    try {
      th.emplace_back([&, t] { for (int i = t; i < n; i += threads) f(i); });
    } catch (...) {
      break;
    }
  }
  for (int t = 0; t < threads; t++)
    if (t == 0 || t >= started)
      for (int i = t; i < n; i += threads) f(i);
  for (auto& x : th) x.join();
}

__host__ __device__ inline int64_t tri_index(int N, int k, int r) {
  return (int64_t)k * N - (int64_t)k * (k - 1) / 2 + (r - k);
}

hk_status build_matrix_impl(int N, hk_rational beta, int prec_bits, void* dev_ws, size_t ws_bytes,
                            hipStream_t s, hk_matrix* out, std::vector<MP>* moments);

// kernel launchers (hk_kernels.hip)
struct InstDesc;
struct SweepArgs;
struct DevPtrs {
  ColInfo* cols; int32_t* itemStart;
  int32_t* A; int64_t* Kc; int32_t* C; int32_t* L; int8_t* L8; uint32_t* S; uint32_t* D; int32_t* dinfo;
  int32_t* nC; int32_t* nCs; int32_t* nL; int32_t* X; int32_t* xs; int32_t* flags;
  int32_t* b32C; int32_t* b32L; int32_t* vec;
  int32_t* LT; int32_t* acc; int64_t* kca; int32_t* ub; uint32_t* us; int32_t* wb;
  int32_t* nU; int32_t* nUs; int32_t* dv1; int32_t* dv2; uint32_t* md;
  int32_t* mdinfo; int64_t* dots;
  InstDesc* desc;
  SweepArgs* sargs;   // the solve arguments of this matrix (hk_solve)
};
DevPtrs dev_ptrs(const Plan& P, char* ws);

// Device descriptor of one instance (one factorisation problem) of a batch;
// every factorisation kernel takes an array of them, a single matrix is a
// batch of one.
struct InstDesc {
  const ColInfo* cols; const int32_t* itemStart;
  int32_t* A; int64_t* Kc; int32_t* C; uint32_t* S; int32_t* L; int8_t* L8; int32_t* LT; uint32_t* D;
  int32_t* dinfo; int32_t* nC; int32_t* nCs; int32_t* nL; int32_t* b32C; int32_t* flags;
  const int32_t* X; const int32_t* xs;
  int32_t N, h, WX, active;
};
InstDesc make_desc(const Plan& P, const DevPtrs& D);

// Host view of a batch: the device descriptor array and the plans (grid sizes
// are computed on the host from the plans).
struct BatchView {
  const InstDesc* ddesc = nullptr;
  std::vector<const Plan*> plans;
  int maxN = 0;
  int ipw = 4;   // update items (wavefronts) per workgroup of k_update / k_update_near: 1, 2 or 4
  int mma = 1;   // bulk updates on the matrix cores where they fit (k_update_mma)
};
extern thread_local std::string g_err;

hipError_t launch_fill32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill64(int64_t* p, int64_t n, hipStream_t s);
hipError_t launch_expand(const BatchView& B, hipStream_t s);
// j = 0: trailing update after the panel [pc, pc + b); j > 0: in-panel
// (left-looking) update of column pc + j by columns [pc, pc + j);
// UPD_NEAR / UPD_FAR: the trailing update split into the next panel's columns
// [pc + b, pc + 2b) and the rest (look-ahead)
constexpr int UPD_NEAR = -1, UPD_FAR = -2;
// the launches of k_update (the bulk of the update work: j = 0 and UPD_FAR)
// against those of k_update_near (in-panel and UPD_NEAR, critical path)
__host__ __device__ inline bool update_is_bulk(int j) { return j == 0 || j == UPD_FAR; }
// widest column of the batch when its bulk updates run on the matrix cores
// (k_update_mma), 0 when they run on the vector units (k_update)
int mma_width(const BatchView& B, int b);
hipError_t launch_update(const BatchView& B, int pc, int b, int j, int rd, hipStream_t s,
                         hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_fdiv(const BatchView& B, int c, int rd, hipStream_t s);
// LDS per workgroup that the current device allows
size_t device_lds_limit();
// empty when every column launch of a factorisation in look-ahead mode `mode`
// fits the device's LDS, else a message naming the first column that does not
std::string factor_lds_check(const BatchView& B, int mode);
hipError_t launch_column(const BatchView& B, int c, hipStream_t s, hipEvent_t t0 = nullptr,
                         hipEvent_t t1 = nullptr);
hipError_t launch_gather_pivots_b(const BatchView& B, int32_t* out, int ld, hipStream_t s);
int64_t update_items(const Plan& P, int pc, int b, int j);
// One factorisation of every instance of B, enqueued on s.  With a second
// stream s2 (may be null) the trailing update of each panel is split: the
// next panel's columns are updated on s, on the critical path, the rest on
// s2 concurrently with the next panel (look-ahead); s2 is joined into s at
// the end.  evs: optional HIP-event pairs around every update launch.
struct TimedLaunch { hipEvent_t t0, t1; bool bulk; };
hipError_t enqueue_factor(const BatchView& B, int b, int mode, hipStream_t s, hipStream_t s2,
                          std::vector<TimedLaunch>* evs, std::vector<hipEvent_t>* pool, size_t* evi,
                          int* n_update, int* n_bulk = nullptr);
// algorithmic limb MACs of the last factorisation of m: all of them, and the
// share its bulk update launches carried under the schedule (panel b, look-
// ahead mode) it ran with (mode 2: the column launches carry all of it)
hipError_t limb_macs_split(hk_matrix m, int b, int mode, hipStream_t s, double* total, double* bulk);
int effective_lookahead(const hk_matrix_s* m);
hipError_t launch_bits(const Plan& P, const DevPtrs& D, hipStream_t s);
// rigorous inertia of m's current factorisation (hk_certify.cpp): the exact
// pivots piv (h fractional bits) with the radii of the midpoint-radius
// enclosure; margins (N, may be NULL) get log2(|d_k| / radius_k)
hk_status certify_factor(hk_matrix m, hipStream_t s, const std::vector<MP>& piv, int* n_negative,
                         int* certified, double* min_margin, double* margins);

// Everything the solve and inverse-iteration kernels need of one instance;
// the batched launches take a device array of these (one per instance).
struct SweepArgs {
  const ColInfo* cols;
  int N, Npad, VA, nbA, VW, LWT, h, bwd, panel, gbits, K, pad;
  int32_t* acc; int64_t* kc; int32_t* ub; uint32_t* us; int32_t* nU; int32_t* nUs;
  const int32_t* L; const int32_t* LT; const int32_t* nL; int32_t* out; int32_t* flags;
  int32_t* v; int32_t* y; int32_t* wb; const uint32_t* Dd; const int32_t* dinfo;
  int64_t* dots; uint32_t* md; int32_t* mdinfo;
};
SweepArgs make_sweep_args(const Plan& P, const DevPtrs& D, int panel, int gbits);
// launch shapes of a batch (maxima over its instances)
struct SweepShape { int count = 0, maxN = 0, maxVA = 0, maxVW = 0, maxLW = 0; int64_t maxVAN = 0;
                    size_t shm_div = 0, shm_scale = 0; };
SweepShape sweep_shape(const std::vector<const Plan*>& plans);
// empty when every launch of the solve sweeps fits the device's LDS, else why not
std::string solve_lds_check(const SweepShape& sh);
// Batched inverse-iteration steps (hk_kernels.hip):
//   vinit_b  stage 0: acc = v 2^(h+g); stage 1: acc = w 2^h
//   vcol_b   one column step of the forward (bwd 0) or backward (bwd 1) substitution
//   vdivide_b w = RNE(z 2^h / d) per row
//   vdots_b  exact <v, y> and <v, v> as lazy int64 digits (dots)
//   vmax_b   the row of largest |y|: its magnitude normalised (md, mdinfo = nd, sh, row)
//   vscale_b v = RNE(y 2^K / max|y|)
hipError_t launch_vinit_b(const SweepArgs* args, const SweepShape& sh, int stage, hipStream_t s);
// one launch per column step j of a sweep (forward: column j, backward:
// column maxN - 1 - j), with the previous column's update folded in
hipError_t launch_vcol_b(const SweepArgs* args, const SweepShape& sh, int bwd, int j, hipStream_t s);
// a whole solve (forward sweep, diagonal, backward sweep) of every instance:
// rhs in SweepArgs::v, result in SweepArgs::y
hipError_t enqueue_solve(const SweepArgs* args, const SweepShape& sh, hipStream_t s);
hipError_t launch_vdivide_b(const SweepArgs* args, const SweepShape& sh, hipStream_t s);
hipError_t launch_vdots_b(const SweepArgs* args, const SweepShape& sh, hipStream_t s);
hipError_t launch_vmax_b(const SweepArgs* args, const SweepShape& sh, hipStream_t s);
hipError_t launch_vscale_b(const SweepArgs* args, const SweepShape& sh, hipStream_t s);
hipError_t launch_vscale(const Plan& P, const DevPtrs& D, const uint32_t* md, int nd, int sh,
                         int32_t* out, hipStream_t s);

}  // namespace hk

struct hk_matrix_s {
  hk::Plan P;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hk::DevPtrs D;
  std::vector<hk::MP> X;
  std::vector<int32_t> xs_host;
  bool factored = false;
  int panel = 4;
  int timing = 0;
  int n_update = 0;
  double update_ms = 0;
  int n_bulk = 0;            // k_update launches (bulk) of the last hk_factor
  double bulk_ms = 0;        // their summed device time (timing on)
  int32_t flags_host[16];
  int gbits = 0;            // solve guard bits from the actual largest moment
  hk::InstDesc desc_host;
  hk::BatchView B;          // this matrix as a batch of one
  std::vector<hipEvent_t> ev;    // per-launch timing and eager look-ahead points
  std::vector<hipEvent_t> gev;   // look-ahead points of the captured graph
  // the launch sequence of one factorisation, captured once per panel width
  // and replayed by hk_factor when per-launch timing is off
  hipStream_t gcap = nullptr, gcap2 = nullptr, s2 = nullptr;   // capture streams; look-ahead stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int gpanel = 0, gla = -1, gipw = 0, gmma = -1, g_nupdate = 0, g_nbulk = 0;
  hk::SweepArgs sweep;        // host copy of the solve arguments (kept alive for the upload)
  hipGraph_t sgraph = nullptr;   // one captured solve, replayed by hk_solve
  hipGraphExec_t sgexec = nullptr;
  int lookahead = -1;       // -1: chosen by size, else the look-ahead mode 0 / 1 / 2
  bool eager = false;       // launch on the caller's stream only: no graph capture, no
                            // second stream (look-ahead mode 1 runs as mode 0)
};

