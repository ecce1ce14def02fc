// Inverse iteration for every instance of a batch at once (not in the
// paper): each instance on its own factorisation of M - sigma I, all of them
// stepped together.  One iteration (right-hand side into the accumulators,
// forward substitution one launch per column, diagonal division, second
// initialisation, backward substitution, the exact dots <v,y> and <v,v>, the
// row of largest |y|, v <- RNE(y 2^K / max|y|)) is a fixed launch sequence
// in which every launch covers all instances; it is captured once as a HIP
// graph and replayed.  The host reads the dots, forms
// lambda = sigma + <v,v> 2^g / <v,y> per instance and stops an instance by
// the same rules as the single-instance iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "hk_batch.hpp"

namespace hk {

namespace {

hk_status bfail(hk_status st, const std::string& msg) { g_err = msg; return st; }

// value of lazy signed int64 digits sum_p d[p] 2^(29 p)
MP lazy64_to_mp(const int64_t* d, int n) {
  const size_t nw = (size_t)(((int64_t)n * DB + 64) / 32 + 4);
  std::vector<uint32_t> pw(nw, 0u), nwv(nw, 0u);
  for (int p = 0; p < n; p++) {
    const int64_t x = d[p];
    if (!x) continue;
    const uint64_t m = x < 0 ? (uint64_t)(-(x + 1)) + 1 : (uint64_t)x;
    std::vector<uint32_t>& w = x < 0 ? nwv : pw;
    const int64_t pos = (int64_t)p * DB;
    unsigned __int128 v = (unsigned __int128)m << (pos & 31);
    uint64_t c = 0;
    for (size_t k = (size_t)(pos >> 5); v != 0 || c != 0; k++) {
      const uint64_t t = (uint64_t)(uint32_t)v + w[k] + c;
      w[k] = (uint32_t)t;
      c = t >> 32;
      v >>= 32;
    }
  }
  MP a, b;
  a.d = pw;
  a.trim();
  b.d = nwv;
  b.trim();
  return sub(a, b);
}

// one inverse-iteration step for every instance, in launch order: the solve
// (right-hand side, forward sweep one launch per column, diagonal, second
// right-hand side, backward sweep), dots, largest row, normalisation
hipError_t enqueue_iteration(const SweepArgs* da, const SweepShape& sh, hipStream_t s) {
  hipError_t e = enqueue_solve(da, sh, s);
  if (e == hipSuccess) e = launch_vdots_b(da, sh, s);
  if (e == hipSuccess) e = launch_vmax_b(da, sh, s);
  if (e == hipSuccess) e = launch_vscale_b(da, sh, s);
  return e;
}

struct GraphHolder {
  hipStream_t cap = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  ~GraphHolder() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

}  // namespace

hk_status batch_inverse(Batch& bt, const std::vector<MP>& sigma, const std::vector<int>& act, int tol,
                        int max_iter, hipStream_t s, std::vector<MP>& lam, std::vector<hk_status>& st,
                        std::vector<int>& iters, double& t_solve) {
  const int count = bt.count;
  lam.assign(count, MP());
  st.assign(count, HK_OK);
  iters.assign(count, 0);
  std::vector<SweepArgs> ha(count);
  std::vector<const Plan*> plans;
  for (int i = 0; i < count; i++) {
    hk_matrix m = bt.mats[i];
    ha[i] = make_sweep_args(m->P, m->D, bt.panel, m->gbits);
    if (!act[i]) ha[i].N = 0;     // nothing to do for this instance
    plans.push_back(&m->P);
  }
  const SweepShape sh = sweep_shape(plans);
  {
    const std::string why = solve_lds_check(sh);
    if (!why.empty()) return bfail(HK_EINVAL, why);
  }
  hipError_t e = hipMemcpyAsync(bt.sargs, ha.data(), sizeof(SweepArgs) * count, hipMemcpyHostToDevice, s);
  // v0 = 1 (K fractional bits) for every active instance; flags cleared
  std::vector<std::vector<int32_t>> v0(count);
  for (int i = 0; i < count && e == hipSuccess; i++) {
    if (!act[i]) continue;
    const Plan& P = bt.mats[i]->P;
    v0[i].assign((size_t)P.N * P.VW, 0);
    const MP one = shl(MP::from_u64(1), P.K);
    for (int r = 0; r < P.N; r++) mp_to_digits(one, v0[i].data() + (size_t)r * P.VW, P.VW);
    e = hipMemcpyAsync(bt.mats[i]->D.dv1, v0[i].data(), sizeof(int32_t) * v0[i].size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fill32(bt.mats[i]->D.flags, 16, 0, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bfail(HK_EDEVICE, std::string("batched inverse setup: ") + hipGetErrorString(e));
  const SweepArgs* da = bt.sargs;
  // one iteration of the whole batch, captured once and replayed
  GraphHolder gh;
  e = hipStreamCreateWithFlags(&gh.cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(gh.cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t ec = enqueue_iteration(da, sh, gh.cap);
    const hipError_t e2 = hipStreamEndCapture(gh.cap, &gh.g);
    e = ec != hipSuccess ? ec : e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&gh.x, gh.g, nullptr, nullptr, 0);
  if (e != hipSuccess) return bfail(HK_EDEVICE, std::string("batched inverse graph: ") + hipGetErrorString(e));
  std::vector<std::vector<int64_t>> dots(count);
  std::vector<std::vector<int32_t>> fl(count, std::vector<int32_t>(16, 0));
  std::vector<MP> lam_prev(count), step_prev(count);
  std::vector<int> have_prev(count, 0), have_step(count, 0), no_shrink(count, 0), open(count, 0);
  int n_open = 0;
  for (int i = 0; i < count; i++) if (act[i]) { open[i] = 1; n_open++; }
  for (int it = 0; it < max_iter && n_open > 0; it++) {
    auto t0 = std::chrono::steady_clock::now();
    e = hipGraphLaunch(gh.x, s);
    for (int i = 0; i < count && e == hipSuccess; i++) {
      if (!open[i]) continue;
      const Plan& P = bt.mats[i]->P;
      dots[i].resize((size_t)4 * DOT_PARTS * (2 * P.VW + 8));
      e = hipMemcpyAsync(dots[i].data(), bt.mats[i]->D.dots, sizeof(int64_t) * dots[i].size(),
                         hipMemcpyDeviceToHost, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(fl[i].data(), bt.mats[i]->D.flags, sizeof(int32_t) * 16, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    t_solve += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (e != hipSuccess) return bfail(HK_EDEVICE, std::string("batched inverse iteration: ") + hipGetErrorString(e));
    for (int i = 0; i < count; i++) {
      if (!open[i]) continue;
      iters[i]++;
      const Plan& P = bt.mats[i]->P;
      const int K = P.K, g = bt.mats[i]->gbits;
      auto close = [&](hk_status r) { st[i] = r; open[i] = 0; n_open--; };
      if (fl[i][0]) { close(HK_EPRECISION); continue; }
      const int np = 2 * P.VW + 8;
      // each dot: DOT_PARTS parts of a row of low parts and a row of high parts
      MP vy, vv;
      for (int r = 0; r < 2 * DOT_PARTS; r++) {
        vy = add(vy, lazy64_to_mp(dots[i].data() + (size_t)r * np, np));
        vv = add(vv, lazy64_to_mp(dots[i].data() + (size_t)(2 * DOT_PARTS + r) * np, np));
      }
      if (vy.sign() <= 0) { close(HK_EPRECISION); continue; }
      const int64_t F = 2 * (int64_t)K + 64;
      const MP lamF = add(shl(sigma[i], F - K), floor_div(shl(vv, g + F), vy));
      if (have_prev[i]) {
        MP stp = sub(lamF, lam_prev[i]);
        stp.neg = false;
        MP lf = lamF;
        lf.neg = false;
        bool stop = false;
        {
          MP lhs = mul(stp, pow10((uint32_t)tol));
          stop = cmp(lhs, lf) <= 0;
        }
        if (!stop && have_step[i]) {
          MP lhs = mul(stp, pow10((uint32_t)(tol / 2)));
          if (cmp(lhs, lf) <= 0 && cmp(stp, step_prev[i]) >= 0) {
            if (++no_shrink[i] >= 2) stop = true;
          } else {
            no_shrink[i] = 0;
          }
        }
        if (stop) {
          lam[i] = rne_shr(lamF, F - K);
          close(HK_OK);
          continue;
        }
        step_prev[i] = stp;
        have_step[i] = 1;
      }
      lam_prev[i] = lamF;
      have_prev[i] = 1;
    }
  }
  for (int i = 0; i < count; i++)
    if (open[i]) st[i] = bfail(HK_ENOCONV, "inverse iteration did not converge");
  return HK_OK;
}

}  // namespace hk
