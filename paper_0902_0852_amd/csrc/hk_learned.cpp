// Learned precision and shift (not in the paper).  The precision-proposal
// network predicts, per instance, the bits the fixed-point factorisation
// needs and ln lambda_1; the proposal is accepted only when the method
// itself agrees with it:
//   * b = proposed bits, sigma = exp(predicted ln lambda_1 - 3 RMSE);
//   * factor M - sigma I at b and at ceil(1.25 b) (one batched graph launch
//     for every instance at both precisions); a pivot <= 0 means sigma is
//     not below lambda_1, and sigma is halved (at most three times, then 0);
//   * inverse iteration on each factorisation; accept lambda(1.25 b) when it
//     agrees with lambda(b) to 10^-digits;
//   * otherwise raise the precision by 1.25 again (at most twice), comparing
//     with the previous level, and fall back to the plain method (inverse
//     iteration at the caller's precision with the inertia bracket) when
//     nothing agrees or the next level would exceed the caller's precision.
// Also: the inertia bracket of many instances at once (the labels the
// network is trained on), and the network's forward pass turned into
// proposals.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hk_batch.hpp"

using namespace hk;

namespace {

hk_status lfail(hk_status st, const std::string& msg) { g_err = msg; return st; }

int even_bits(double b) {
  int64_t k = (int64_t)std::ceil(b);
  k = std::max<int64_t>(k, 64);
  k = (k + 31) / 32 * 32;   // whole 32-bit words
  return (int)std::min<int64_t>(k, 1 << 24);
}

// sigma 2^K as an integer from ln sigma (0 when it underflows K bits)
MP fixed_from_log(double ln_sigma, int K) {
  const double t = ln_sigma / std::log(2.0) + K;   // log2(sigma 2^K)
  if (!std::isfinite(t) || t < 0) return MP();
  const int64_t ip = (int64_t)std::floor(t);
  const double frac = t - (double)ip;
  const uint64_t mant = (uint64_t)std::ldexp(std::exp2(frac), 52);   // in [2^52, 2^53)
  MP m = MP::from_u64(mant);
  return ip >= 52 ? shl(m, ip - 52) : shr_mag(m, 52 - ip);
}

struct Entry {
  int inst;          // index into the caller's instances
  int K;
  MP sigma;          // K fractional bits
  int halvings = 0;
  MP lam;            // K fractional bits
  hk_status st = HK_OK;
  int solves = 0;
  int factorizations = 0;
};

// factor every entry at its shift (halving shifts that are not below
// lambda_1), then inverse iteration on each; fills lam / st
hk_status run_entries(std::vector<Entry>& E, const hk_instance* inst, int digits, int panel, void* ws,
                      size_t ws_bytes, hipStream_t s, int& graph_launches) {
  const int n = (int)E.size();
  std::vector<hk_instance> bi(n);
  for (int j = 0; j < n; j++) {
    bi[j] = inst[E[j].inst];
    bi[j].prec_bits = E[j].K;
  }
  Batch bt;
  hk_status st = build_batch(bt, bi.data(), n, ws, ws_bytes, s);
  if (st != HK_OK) return st;
  {
    const Schedule sc = tuned_schedule(bi.data(), n);
    bt.panel = panel > 0 ? panel : (sc.panel > 0 ? sc.panel : 4);
    bt.lookahead = sc.lookahead;
  }
  std::vector<MP> x(n);
  std::vector<int> act(n, 1);
  for (int j = 0; j < n; j++) x[j] = E[j].sigma;
  std::vector<BEval> ev;
  for (int attempt = 0; attempt < 5; attempt++) {
    st = factor_batch(bt, x, act, s, ev, false);
    if (st != HK_OK) return st;
    bool again = false;
    for (int j = 0; j < n; j++) {
      if (!act[j]) continue;
      E[j].factorizations++;
      // any pivot <= 0 (the last one included) means sigma is not below lambda_1
      const bool above = ev[j].st == HK_ENOTSPD || (ev[j].st == HK_OK && ev[j].first_bad >= 0);
      if (above && !x[j].is_zero()) {
        x[j] = E[j].halvings < 3 ? shr_mag(x[j], 1) : MP();
        E[j].halvings++;
        again = true;
      } else {
        act[j] = 0;
        E[j].st = above ? HK_ENOTSPD : ev[j].st;
      }
    }
    if (!again) break;
  }
  graph_launches += bt.graph_launches;
  // factor_batch left each factor in place; inverse iteration on all of them
  std::vector<int> ok(n, 0);
  for (int j = 0; j < n; j++) {
    E[j].sigma = x[j];
    ok[j] = E[j].st == HK_OK;
  }
  std::vector<MP> lam;
  std::vector<hk_status> ist;
  std::vector<int> iters;
  double ts = 0;
  st = batch_inverse(bt, x, ok, digits + 1, 80, s, lam, ist, iters, ts);
  if (st != HK_OK) return st;
  for (int j = 0; j < n; j++) {
    if (!ok[j]) continue;
    E[j].st = ist[j];
    E[j].lam = lam[j];
    E[j].solves = iters[j];
  }
  return HK_OK;
}

}  // namespace

extern "C" {

size_t hk_learned_workspace_bytes(const hk_instance* inst, int count, const int* bits_hat) {
  if (!inst || !bits_hat || count < 1) return 0;
  // pass 0: every instance at b and 1.25 b; escalations: at most every
  // instance once more, at a precision <= 1.25^3 b (capped by prec_bits);
  // fallback: one instance at a time at prec_bits
  std::vector<hk_instance> first, later;
  for (int i = 0; i < count; i++) {
    const int b = even_bits(bits_hat[i]);
    const int b2 = even_bits(1.25 * b);
    if (b2 > inst[i].prec_bits) continue;
    hk_instance a = inst[i];
    a.prec_bits = b;
    first.push_back(a);
    a.prec_bits = b2;
    first.push_back(a);
    a.prec_bits = std::min(inst[i].prec_bits, even_bits(1.25 * even_bits(1.25 * b2)));
    later.push_back(a);
  }
  size_t need = 0;
  if (!first.empty()) {
    need = std::max(batch_bytes(first.data(), (int)first.size()), batch_bytes(later.data(), (int)later.size()));
    if (need == 0) return 0;
  }
  for (int i = 0; i < count; i++) {
    const size_t one = hk_workspace_bytes(inst[i].N, inst[i].beta, inst[i].prec_bits, 0);
    if (one == 0) return 0;
    need = std::max(need, one);
  }
  return need;
}

hk_status hk_bracket_batched(const hk_instance* inst, int count, const char* const* lambda_dec, int digits,
                             int panel, void* dev_ws, size_t ws_bytes, hipStream_t s, int* ok) {
  if (!inst || !lambda_dec || !ok || count < 1) return lfail(HK_EINVAL, "bad arguments");
  if (digits < 2 || digits > 150) return lfail(HK_EINVAL, "digits must be in [2, 150]");
  std::vector<MP> xlo(count), xhi(count);
  for (int i = 0; i < count; i++) {
    MP D;
    int64_t e;
    if (!parse_decimal(lambda_dec[i], digits, D, e))
      return lfail(HK_EINVAL, "instance " + std::to_string(i) + ": malformed decimal");
    xlo[i] = decimal_to_fixed(D, e, inst[i].prec_bits, false);
    xhi[i] = decimal_to_fixed(add(D, MP::from_u64(1)), e, inst[i].prec_bits, true);
  }
  Batch bt;
  hk_status st = build_batch(bt, inst, count, dev_ws, ws_bytes, s);
  if (st != HK_OK) return st;
  {
    const Schedule sc = tuned_schedule(inst, count);
    bt.panel = panel > 0 ? panel : (sc.panel > 0 ? sc.panel : 4);
    bt.lookahead = sc.lookahead;
    if (sc.ipw > 0) bt.B.ipw = sc.ipw;
    if (sc.mma >= 0) bt.B.mma = sc.mma;
  }
  std::vector<int> act(count, 1);
  std::vector<BEval> elo, ehi;
  st = factor_batch(bt, xlo, act, s, elo, false);
  if (st == HK_OK) st = factor_batch(bt, xhi, act, s, ehi, false);
  if (st != HK_OK) return st;
  for (int i = 0; i < count; i++) {
    const int N = inst[i].N;
    ok[i] = elo[i].st == HK_OK && elo[i].nneg == 0 && elo[i].first_bad < 0 && ehi[i].st == HK_OK &&
            ehi[i].nneg == 1 && ehi[i].first_bad == N - 1;
  }
  return HK_OK;
}

hk_status hk_mlp_propose(const float* dev_W, const hk_mlp_meta* meta, const hk_instance* inst, int count,
                         float* dev_io, hipStream_t s, int* bits_hat, double* ln_sigma_hat) {
  if (!dev_W || !meta || !inst || !dev_io || !bits_hat || !ln_sigma_hat || count < 1)
    return lfail(HK_EINVAL, "bad arguments");
  std::vector<float> X(3 * (size_t)count), Y(2 * (size_t)count);
  for (int i = 0; i < count; i++) {
    if (inst[i].N < 1 || inst[i].beta.num < 1 || inst[i].beta.den < 1) return lfail(HK_EINVAL, "bad instance");
    const double f[3] = {(double)inst[i].N, (double)inst[i].beta.num / (double)inst[i].beta.den,
                         std::log((double)inst[i].N)};
    for (int k = 0; k < 3; k++) X[3 * i + k] = (float)((f[k] - meta->in_mean[k]) / meta->in_scale[k]);
  }
  hipError_t e = hipMemcpyAsync(dev_io, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return lfail(HK_EDEVICE, hipGetErrorString(e));
  hk_status st = hk_mlp_forward(dev_W, dev_io, count, dev_io + 3 * count, nullptr, s);
  if (st != HK_OK) return st;
  e = hipMemcpyAsync(Y.data(), dev_io + 3 * count, sizeof(float) * Y.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return lfail(HK_EDEVICE, hipGetErrorString(e));
  for (int i = 0; i < count; i++) {
    const double bits = (double)Y[2 * i] * meta->out_scale[0] + meta->out_mean[0];
    const double lnl = (double)Y[2 * i + 1] * meta->out_scale[1] + meta->out_mean[1];
    bits_hat[i] = even_bits(std::max(64.0, bits * meta->bits_margin));
    ln_sigma_hat[i] = lnl - 3.0 * meta->rmse_ln_lambda;
  }
  return HK_OK;
}

hk_status hk_eig_learned(const hk_instance* inst, int count, const int* bits_hat, const double* ln_sigma_hat,
                         int digits, int panel, void* dev_ws, size_t ws_bytes, hipStream_t s, hk_result* out,
                         hk_batch_report* rep) {
  auto t0 = std::chrono::steady_clock::now();
  if (!inst || !bits_hat || !ln_sigma_hat || !out || count < 1) return lfail(HK_EINVAL, "bad arguments");
  if (digits < 2 || digits > 150) return lfail(HK_EINVAL, "digits must be in [2, 150]");
  const size_t need = hk_learned_workspace_bytes(inst, count, bits_hat);
  if (need == 0) return HK_EINVAL;
  if (!dev_ws || ws_bytes < need) return lfail(HK_EINVAL, "workspace too small: need " + std::to_string(need));
  int graph_launches = 0;
  std::vector<int> done(count, 0), level(count, 0), total_solves(count, 0), nfact(count, 0);
  std::vector<MP> prev(count);      // lambda at the previous level
  std::vector<int> prevK(count, 0);
  for (int i = 0; i < count; i++) memset(&out[i], 0, sizeof(hk_result));
  // levels: b, 1.25 b, 1.25^2 b, ...; each round computes the next level for
  // every instance still open and compares it with the level before
  std::vector<Entry> E;
  for (int i = 0; i < count; i++) {
    const int b = even_bits(bits_hat[i]);
    if (even_bits(1.25 * b) > inst[i].prec_bits) continue;
    for (int k = 0; k < 2; k++) {
      Entry en;
      en.inst = i;
      en.K = k == 0 ? b : even_bits(1.25 * b);
      en.sigma = fixed_from_log(ln_sigma_hat[i], en.K);
      E.push_back(en);
    }
  }
  hk_status st = HK_OK;
  for (int round = 0; round < 3 && !E.empty(); round++) {
    st = run_entries(E, inst, digits, panel, dev_ws, ws_bytes, s, graph_launches);
    if (st != HK_OK) return st;
    std::vector<Entry> next;
    for (size_t j = 0; j < E.size(); j++) {
      const Entry& en = E[j];
      const int i = en.inst;
      total_solves[i] += en.solves;
      nfact[i] += en.factorizations;
      if (round == 0 && (j % 2) == 0) {
        // the first level of this instance: keep it for the comparison
        if (en.st == HK_OK) { prev[i] = en.lam; prevK[i] = en.K; }
        continue;
      }
      bool accepted = false;
      if (en.st == HK_OK && prevK[i] > 0) {
        const MP a = shl(prev[i], en.K - prevK[i]);
        accepted = agree(a, en.lam, digits);
      }
      if (accepted) {
        done[i] = 1;
        out[i].status = HK_OK;
        out[i].path = 1;
        out[i].bits_used = en.K;
        snprintf(out[i].lambda_dec, sizeof out[i].lambda_dec, "%s", decimal_string(en.lam, en.K, digits + 5).c_str());
        lambda_mpf(en.lam, en.K, &out[i].lambda, out[i].lambda_words);
        continue;
      }
      // raise the precision once more, relative to this level
      if (en.st == HK_OK) { prev[i] = en.lam; prevK[i] = en.K; }
      const int K2 = even_bits(1.25 * en.K);
      if (round < 2 && K2 <= inst[i].prec_bits) {
        Entry nx;
        nx.inst = i;
        nx.K = K2;
        nx.sigma = shl(en.sigma, K2 - en.K);   // the shift that worked at this level
        next.push_back(nx);
      }
    }
    E.swap(next);
  }
  // fallback: the plain method at the caller's precision, one instance at a time
  hk_status first = HK_OK;
  for (int i = 0; i < count; i++) {
    if (!done[i]) {
      hk_report r;
      char dec[192];
      hk_status si = hk_smallest_eig(inst[i].N, inst[i].beta, inst[i].prec_bits, HK_INVERSE | HK_FLAG_NO_WORK_COUNT,
                                     digits + 5, nullptr, dev_ws, ws_bytes, s, dec, sizeof dec, &r);
      out[i].status = si;
      out[i].path = 0;
      out[i].bits_used = inst[i].prec_bits;
      out[i].verified = r.verified;
      total_solves[i] += r.solves;
      nfact[i] += r.factorizations;
      snprintf(out[i].lambda_dec, sizeof out[i].lambda_dec, "%s", dec);
      out[i].lambda = r.lambda;
      memcpy(out[i].lambda_words, r.lambda_words, sizeof r.lambda_words);
      out[i].lambda.digits = out[i].lambda_words;
    }
    out[i].solves = total_solves[i];
    out[i].factorizations = nfact[i];
    if (first == HK_OK && out[i].status != HK_OK) first = out[i].status;
  }
  if (rep) {
    rep->panel = panel;
    rep->graph_launches = graph_launches;
    rep->t_build_s = 0;
    rep->t_factor_s = 0;
    rep->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (first != HK_OK) g_err = "some instances failed";
  return first;
}

}  // extern "C"
