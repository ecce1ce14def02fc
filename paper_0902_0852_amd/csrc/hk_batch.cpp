// Batched form: many instances factored together by instance-batched
// kernels, one factorisation captured as a HIP graph and replayed; the
// paper's Secant iteration per instance in lockstep, then the inertia
// bracket.  See include/hk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "hk_batch.hpp"

using namespace hk;

namespace hk {

hk_status dfail_b(hk_status st, const std::string& msg) { g_err = msg; return st; }

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

Batch::~Batch() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (cap) (void)hipStreamDestroy(cap);
  if (cap2) (void)hipStreamDestroy(cap2);
  if (s2) (void)hipStreamDestroy(s2);
  for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : tevents) (void)hipEventDestroy(ev);
  for (size_t i = (size_t)borrowed; i < mats.size(); i++) hk_matrix_destroy(mats[i]);
}

// per-batch layout: descriptors, flags, pivot rows, then one workspace per instance
static bool batch_layout(const hk_instance* inst, int count, std::vector<size_t>& off, size_t& total,
                         int& maxN, int& ld) {
  maxN = 0; ld = 0;
  std::vector<size_t> sz(count);
  for (int i = 0; i < count; i++) {
    Plan P;
    std::string err;
    if (!make_plan(inst[i].N, inst[i].beta.num, inst[i].beta.den, inst[i].prec_bits, P, err)) {
      g_err = "instance " + std::to_string(i) + ": " + err;
      return false;
    }
    sz[i] = P.total;
    maxN = std::max(maxN, P.N);
    ld = std::max(ld, P.maxW + WB);
  }
  size_t o = 0;
  o = al256(o + sizeof(InstDesc) * count);
  o = al256(o + sizeof(int32_t) * 16 * count);
  o = al256(o + sizeof(int32_t) * (size_t)count * maxN * ld);
  o = al256(o + sizeof(SweepArgs) * count);
  off.resize(count);
  for (int i = 0; i < count; i++) { off[i] = o; o = al256(o + sz[i]); }
  total = o;
  return true;
}

__global__ void k_reset_flags(int32_t* flags, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count * 16) flags[i] = (i % 16) == 1 ? INT_MAX : 0;
}

hk_status build_batch(Batch& bt, const hk_instance* inst, int count, void* ws, size_t ws_bytes,
                      hipStream_t s) {
  std::vector<size_t> off;
  size_t total;
  if (count < 1) return dfail_b(HK_EINVAL, "empty batch");
  if (!batch_layout(inst, count, off, total, bt.maxN, bt.ld)) return HK_EINVAL;
  if (!ws || ws_bytes < total) return dfail_b(HK_EINVAL, "workspace too small: need " + std::to_string(total));
  char* base = (char*)ws;
  bt.count = count;
  bt.ddesc = (InstDesc*)base;
  bt.flags = (int32_t*)(base + al256(sizeof(InstDesc) * count));
  bt.piv = (int32_t*)((char*)bt.flags + al256(sizeof(int32_t) * 16 * count));
  bt.sargs = (SweepArgs*)((char*)bt.piv + al256(sizeof(int32_t) * (size_t)count * bt.maxN * bt.ld));
  // moments of all instances in parallel host threads
  std::vector<std::vector<MP>> X(count);
  std::vector<int> ok(count, 0);
  {
    const int nth = std::max(1, std::min<int>(count, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nth; t++)
      th.emplace_back([&, t] {
        for (int i = t; i < count; i += nth) {
          uint32_t p, q;
          if (!reduce_beta(inst[i].beta.num, inst[i].beta.den, &p, &q)) continue;
          ok[i] = build_moments(inst[i].N, p, q, inst[i].prec_bits, X[i]) ? 1 : 0;
        }
      });
    for (auto& t : th) t.join();
  }
  for (int i = 0; i < count; i++) {
    if (!ok[i]) return dfail_b(HK_EPRECISION, "moments of instance " + std::to_string(i));
    hk_matrix m = nullptr;
    hk_status st = build_matrix_impl(inst[i].N, inst[i].beta, inst[i].prec_bits, base + off[i],
                                     ws_bytes - off[i], s, &m, &X[i]);
    if (st != HK_OK) return st;
    bt.mats.push_back(m);
    InstDesc d = m->desc_host;
    d.flags = bt.flags + 16 * i;
    bt.hdesc.push_back(d);
    bt.B.plans.push_back(&m->P);
  }
  bt.B.ddesc = bt.ddesc;
  bt.B.maxN = bt.maxN;
  hipError_t e = hipMemcpyAsync(bt.ddesc, bt.hdesc.data(), sizeof(InstDesc) * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dfail_b(HK_EDEVICE, hipGetErrorString(e));
  return HK_OK;
}

// capture (once per panel width) the launch sequence of one factorisation
static hk_status ensure_graph(Batch& bt) {
  int maxW = 0;
  for (const Plan* p : bt.B.plans) maxW = std::max(maxW, p->maxW);
  const int la = lookahead_mode(bt.lookahead, bt.maxN, maxW);
  const std::string why = factor_lds_check(bt.B, la);
  if (!why.empty()) return dfail_b(HK_EINVAL, why);
  if (bt.timing) return HK_OK;   // launched one by one
  if (bt.exec && bt.captured_panel == bt.panel && bt.captured_la == la && bt.captured_ipw == bt.B.ipw &&
      bt.captured_mma == bt.B.mma)
    return HK_OK;
  if (bt.exec) { (void)hipGraphExecDestroy(bt.exec); bt.exec = nullptr; }
  if (bt.graph) { (void)hipGraphDestroy(bt.graph); bt.graph = nullptr; }
  hipError_t e = hipSuccess;
  if (!bt.cap) e = hipStreamCreateWithFlags(&bt.cap, hipStreamNonBlocking);
  if (e == hipSuccess && !bt.cap2 && la == 1) e = hipStreamCreateWithFlags(&bt.cap2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(bt.cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_reset_flags, dim3((bt.count * 16 + 255) / 256), dim3(256), 0, bt.cap, bt.flags,
                       bt.count);
    e = hipGetLastError();
    size_t evi = 0;
    if (e == hipSuccess)
      e = enqueue_factor(bt.B, bt.panel, la, bt.cap, la == 1 ? bt.cap2 : nullptr, nullptr, &bt.events, &evi,
                         nullptr);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(bt.cap, &g);
    if (e == hipSuccess) e = e2;
    bt.graph = g;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&bt.exec, bt.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return dfail_b(HK_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  bt.captured_panel = bt.panel;
  bt.captured_la = la;
  bt.captured_ipw = bt.B.ipw;
  bt.captured_mma = bt.B.mma;
  return HK_OK;
}

hk_status factor_batch(Batch& bt, const std::vector<MP>& x, const std::vector<int>& act, hipStream_t s,
                       std::vector<BEval>& out, bool want_pivots) {
  hk_status st = ensure_graph(bt);
  if (st != HK_OK) return st;
  std::vector<std::vector<int32_t>> xs(bt.count);
  hipError_t e = hipSuccess;
  for (int i = 0; i < bt.count && e == hipSuccess; i++) {
    bt.hdesc[i].active = act[i];
    if (!act[i]) continue;
    const Plan& P = bt.mats[i]->P;
    xs[i].assign(P.WX, 0);
    mp_to_digits(x[i], xs[i].data(), P.WX);
    if (x[i].bitlen() > (int64_t)(P.WX - 2) * DB) return dfail_b(HK_EINVAL, "shift too wide");
    e = hipMemcpyAsync(bt.mats[i]->D.xs, xs[i].data(), sizeof(int32_t) * P.WX, hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(bt.ddesc, bt.hdesc.data(), sizeof(InstDesc) * bt.count, hipMemcpyHostToDevice, s);
  std::vector<TimedLaunch> evs;
  if (e == hipSuccess && bt.timing) {
    int maxW = 0;
    for (const Plan* p : bt.B.plans) maxW = std::max(maxW, p->maxW);
    const int la = lookahead_mode(bt.lookahead, bt.maxN, maxW);
    if (!bt.s2 && la == 1) e = hipStreamCreateWithFlags(&bt.s2, hipStreamNonBlocking);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_reset_flags, dim3((bt.count * 16 + 255) / 256), dim3(256), 0, s, bt.flags, bt.count);
      e = hipGetLastError();
    }
    size_t evi = 0;
    int nu = 0, nbk = 0;
    if (e == hipSuccess)
      e = enqueue_factor(bt.B, bt.panel, la, s, la == 1 ? bt.s2 : nullptr, &evs, &bt.tevents, &evi, &nu, &nbk);
    bt.n_update += nu;
    bt.n_bulk += nbk;
  } else if (e == hipSuccess) {
    e = hipGraphLaunch(bt.exec, s);
  }
  bt.graph_launches++;
  std::vector<int32_t> fl(16 * bt.count);
  std::vector<int32_t> pv;
  if (e == hipSuccess && want_pivots) {
    e = launch_gather_pivots_b(bt.B, bt.piv, bt.ld, s);
    pv.resize((size_t)bt.count * bt.maxN * bt.ld);
    if (e == hipSuccess) e = hipMemcpyAsync(pv.data(), bt.piv, sizeof(int32_t) * pv.size(), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(fl.data(), bt.flags, sizeof(int32_t) * fl.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (size_t k = 0; k < evs.size() && e == hipSuccess; k++) {
    float ms = 0;
    e = hipEventElapsedTime(&ms, evs[k].t0, evs[k].t1);
    bt.update_ms += ms;
    if (evs[k].bulk) bt.bulk_ms += ms;
  }
  if (e != hipSuccess) return dfail_b(HK_EDEVICE, std::string("batched factorisation: ") + hipGetErrorString(e));
  out.assign(bt.count, BEval());
  for (int i = 0; i < bt.count; i++) {
    if (!act[i]) continue;
    const int N = bt.mats[i]->P.N;
    BEval& ev = out[i];
    const int32_t* f = &fl[16 * i];
    ev.first_bad = f[1] == INT_MAX ? -1 : f[1];
    ev.nneg = f[2];
    ev.st = f[0] ? HK_EPRECISION : ((ev.first_bad >= 0 && ev.first_bad < N - 1) ? HK_ENOTSPD : HK_OK);
    bt.mats[i]->factored = ev.st == HK_OK;
    if (want_pivots && ev.st == HK_OK) ev.piv.resize(N);
  }
  if (want_pivots) {
    // pivots to host integers, every instance's at once on the host threads
    std::vector<std::pair<int, int>> jobs;
    for (int i = 0; i < bt.count; i++)
      for (int k = 0; k < (int)out[i].piv.size(); k++) jobs.emplace_back(i, k);
    parallel_for((int)jobs.size(), std::min(host_threads(), (int)jobs.size() / 64), [&](int t) {
      const int i = jobs[t].first, k = jobs[t].second;
      out[i].piv[k] = digits_to_mp(pv.data() + ((size_t)i * bt.maxN + k) * bt.ld, bt.ld, 1);
    });
  }
  return HK_OK;
}

static std::string tune_key(const hk_instance* inst, int count) {
  int maxN = 0, maxK = 0;
  for (int i = 0; i < count; i++) { maxN = std::max(maxN, inst[i].N); maxK = std::max(maxK, inst[i].prec_bits); }
  int nb = 1, kb = 1;
  while (nb < maxN) nb <<= 1;
  while (kb < maxK) kb <<= 1;
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
  }
  std::ostringstream os;
  os << arch << " count=" << count << " N<=" << nb << " K<=" << kb;
  return os.str();
}

static Schedule cached_schedule(const std::string& key) {
  Schedule sc;
  const char* path = getenv("HK_TUNE_CACHE");
  if (!path) return sc;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t bar = line.find(" | panel=");
    if (bar == std::string::npos || line.substr(0, bar) != key) continue;
    sc.panel = atoi(line.c_str() + bar + 9);
    const size_t la = line.find(" la=", bar);
    sc.lookahead = la == std::string::npos ? -1 : atoi(line.c_str() + la + 4);
    const size_t ip = line.find(" ipw=", bar);
    sc.ipw = ip == std::string::npos ? 0 : atoi(line.c_str() + ip + 5);
    const size_t mm = line.find(" mma=", bar);
    sc.mma = mm == std::string::npos ? -1 : atoi(line.c_str() + mm + 5);
  }
  return sc;
}

// the paper's Secant iteration is reused from hk_drivers.cpp through this
// interface (one machine per instance)
struct SecantRun;
SecantRun* secant_new(int N, int K, int h, int tol, int max_eval);
void secant_delete(SecantRun* r);
void secant_threads(SecantRun* r, int threads);
bool secant_next(SecantRun* r, MP& x, int& inertia);
bool secant_start_pair(SecantRun* r, MP& x0, MP& x1);
void secant_feed(SecantRun* r, hk_status st, int nneg, int first_bad, std::vector<MP>&& piv);
bool secant_done(SecantRun* r, MP& lam, hk_status& st, std::string& err);

// the paired batch's own part: descriptors, flags, pivot rows and solve
// arguments for 2 count instances, then a second workspace per instance (the
// sizes of the batch's own)
static bool twin_layout(const hk_instance* inst, int count, std::vector<size_t>& off2, size_t& total2) {
  std::vector<size_t> off;
  size_t total;
  int maxN, ld;
  if (!batch_layout(inst, count, off, total, maxN, ld)) return false;
  size_t o = 0;
  o = al256(o + sizeof(InstDesc) * 2 * count);
  o = al256(o + sizeof(int32_t) * 16 * 2 * count);
  o = al256(o + sizeof(int32_t) * (size_t)2 * count * maxN * ld);
  o = al256(o + sizeof(SweepArgs) * 2 * count);
  off2.resize(count);
  for (int i = 0; i < count; i++) {
    off2[i] = o;
    o = al256(o + ((i + 1 < count ? off[i + 1] : total) - off[i]));
  }
  total2 = o;
  return true;
}

size_t twin_bytes(const hk_instance* inst, int count) {
  std::vector<size_t> off2;
  size_t total2;
  if (!inst || count < 1 || !twin_layout(inst, count, off2, total2)) return 0;
  return total2;
}

hk_status build_twin(Batch& tw, Batch& bt, const hk_instance* inst, int count, void* ws, size_t ws_bytes,
                     hipStream_t s) {
  std::vector<size_t> off2;
  size_t total2;
  if (!twin_layout(inst, count, off2, total2)) return HK_EINVAL;
  if (!ws || ws_bytes < total2) return dfail_b(HK_EINVAL, "paired workspace too small");
  char* base = (char*)ws;
  tw.count = 2 * count;
  tw.maxN = bt.maxN;
  tw.ld = bt.ld;
  tw.ddesc = (InstDesc*)base;
  tw.flags = (int32_t*)(base + al256(sizeof(InstDesc) * 2 * count));
  tw.piv = (int32_t*)((char*)tw.flags + al256(sizeof(int32_t) * 16 * 2 * count));
  tw.sargs = (SweepArgs*)((char*)tw.piv + al256(sizeof(int32_t) * (size_t)2 * count * tw.maxN * tw.ld));
  tw.borrowed = count;
  for (int i = 0; i < 2 * count; i++) {
    hk_matrix m = nullptr;
    if (i < count) {
      m = bt.mats[i];
    } else {
      const int j = i - count;
      std::vector<MP> X = bt.mats[j]->X;   // the moments are the batch's own
      hk_status st = build_matrix_impl(inst[j].N, inst[j].beta, inst[j].prec_bits, base + off2[j],
                                       ws_bytes - off2[j], s, &m, &X);
      if (st != HK_OK) return st;
    }
    tw.mats.push_back(m);
    InstDesc d = m->desc_host;
    d.flags = tw.flags + 16 * i;
    tw.hdesc.push_back(d);
    tw.B.plans.push_back(&m->P);
  }
  tw.B.ddesc = tw.ddesc;
  tw.B.maxN = tw.maxN;
  tw.B.ipw = bt.B.ipw;
  tw.B.mma = bt.B.mma;
  tw.panel = bt.panel;
  tw.lookahead = bt.lookahead;
  tw.timing = bt.timing;
  hipError_t e = hipMemcpyAsync(tw.ddesc, tw.hdesc.data(), sizeof(InstDesc) * 2 * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dfail_b(HK_EDEVICE, hipGetErrorString(e));
  return HK_OK;
}

size_t batch_bytes(const hk_instance* inst, int count) {
  std::vector<size_t> off;
  size_t total;
  int maxN, ld;
  if (!inst || count < 1) return 0;
  if (!batch_layout(inst, count, off, total, maxN, ld)) return 0;
  return total;
}

Schedule tuned_schedule(const hk_instance* inst, int count) { return cached_schedule(tune_key(inst, count)); }

}  // namespace hk

extern "C" {

size_t hk_batch_workspace_bytes(const hk_instance* inst, int count) { return batch_bytes(inst, count); }

size_t hk_batch_workspace_bytes_paired(const hk_instance* inst, int count) {
  const size_t a = batch_bytes(inst, count), b = twin_bytes(inst, count);
  return a && b ? ((a + 255) & ~(size_t)255) + b : 0;
}

hk_status hk_eig_batched(const hk_instance* inst, int count, int digits, int panel, void* dev_ws,
                         size_t ws_bytes, hipStream_t s, hk_result* out, hk_batch_report* rep) {
  auto t0 = std::chrono::steady_clock::now();
  if (!inst || !out || count < 1) return dfail_b(HK_EINVAL, "bad arguments");
  if (digits < 2 || digits > 150) return dfail_b(HK_EINVAL, "digits must be in [2, 150]");
  for (int i = 0; i < count; i++)
    if ((inst[i].method & 0xff) != HK_INVERSE && (inst[i].method & 0xff) != HK_SECANT)
      return dfail_b(HK_EINVAL, "instance " + std::to_string(i) + ": unknown method");
  Batch bt;
  hk_status st = build_batch(bt, inst, count, dev_ws, ws_bytes, s);
  if (st != HK_OK) return st;
  {
    const Schedule sc = tuned_schedule(inst, count);
    bt.panel = panel > 0 ? panel : (sc.panel > 0 ? sc.panel : 4);
    bt.lookahead = sc.lookahead;
    if (sc.ipw > 0) bt.B.ipw = sc.ipw;
    if (sc.mma >= 0) bt.B.mma = sc.mma;
    // the first instance's flags set the schedule of the whole batch
    const int fl = inst[0].method;
    if (fl & HK_FLAG_LOOKAHEAD_ON) bt.lookahead = 1;
    if (fl & HK_FLAG_LOOKAHEAD_OFF) bt.lookahead = 0;
    if (fl & HK_FLAG_LOOKAHEAD_FUSED) bt.lookahead = 2;
    const int g = (fl >> 28) & 7;
    if (g == 1 || g == 2 || g == 4) bt.B.ipw = g;
    if (fl & HK_FLAG_VECTOR_UPDATE) bt.B.mma = 0;
    bt.timing = (fl & HK_FLAG_TIME_UPDATES) != 0;
  }
  // with room for a second copy of every instance, the two start points of
  // the Secant and the two ends of the bracket are factored together
  Batch tw;
  bool paired = false;
  {
    const size_t own = (batch_bytes(inst, count) + 255) & ~(size_t)255, t2 = twin_bytes(inst, count);
    if (t2 > 0 && ws_bytes >= own + t2) {
      st = build_twin(tw, bt, inst, count, (char*)dev_ws + own, ws_bytes - own, s);
      if (st != HK_OK) return st;
      paired = true;
    }
  }
  auto t1 = std::chrono::steady_clock::now();
  std::vector<SecantRun*> sm(count, nullptr);
  for (int i = 0; i < count; i++) {
    const Plan& P = bt.mats[i]->P;
    if ((inst[i].method & 0xff) == HK_SECANT) sm[i] = secant_new(P.N, P.K, P.h, digits, 200);
    memset(&out[i], 0, sizeof(hk_result));
  }
  std::vector<MP> x(count), lam(count);
  std::vector<int> act(count), inertia(count), nfact(count, 0), done(count, 0);
  std::vector<BEval> ev;
  // the paper's Secant iteration, every Secant instance in lockstep
  st = HK_OK;
  // each round's Secant steps of the instances run side by side on the host,
  // the host threads shared out among them
  int nsec = 0;
  for (int i = 0; i < count; i++) nsec += sm[i] ? 1 : 0;
  const int ith = std::min(nsec, host_threads());
  for (int i = 0; i < count; i++)
    if (sm[i]) secant_threads(sm[i], host_threads() / std::max(1, ith));
  if (paired && nsec > 0) {
    // round 0: both start points of every Secant instance in one factorisation
    std::vector<MP> x2(2 * count), xb(count);
    std::vector<int> a2(2 * count, 0);
    for (int i = 0; i < count; i++)
      if (sm[i] && secant_start_pair(sm[i], x2[i], xb[i])) { x2[count + i] = xb[i]; a2[i] = a2[count + i] = 1; }
    st = factor_batch(tw, x2, a2, s, ev, true);
    for (int i = 0; i < count && st == HK_OK; i++) {
      if (!a2[i]) continue;
      MP xs;
      int inert = 0;
      if (!secant_next(sm[i], xs, inert)) continue;
      nfact[i]++;
      secant_feed(sm[i], ev[i].st, ev[i].nneg, ev[i].first_bad, std::move(ev[i].piv));
      if (!secant_next(sm[i], xs, inert) || cmp(xs, xb[i]) != 0) continue;
      nfact[i]++;
      secant_feed(sm[i], ev[count + i].st, ev[count + i].nneg, ev[count + i].first_bad, std::move(ev[count + i].piv));
    }
  }
  for (int round = 0; round < 400 && st == HK_OK; round++) {
    parallel_for(count, ith, [&](int i) { act[i] = sm[i] && secant_next(sm[i], x[i], inertia[i]) ? 1 : 0; });
    bool any = false;
    for (int i = 0; i < count; i++) any |= act[i] != 0;
    if (!any) break;
    st = factor_batch(bt, x, act, s, ev, true);
    for (int i = 0; i < count && st == HK_OK; i++) {
      if (!act[i]) continue;
      nfact[i]++;
      secant_feed(sm[i], ev[i].st, ev[i].nneg, ev[i].first_bad, std::move(ev[i].piv));
    }
  }
  for (int i = 0; i < count && st == HK_OK; i++) {
    if (!sm[i]) continue;
    hk_status si;
    std::string err;
    if (secant_done(sm[i], lam[i], si, err)) done[i] = 1;
    else out[i].status = si;
  }
  // inverse iteration (not in the paper) for the other instances: one
  // factorisation at the shift hint (halved while a pivot is <= 0, at most
  // three times, then 0) or at 0, then all of them stepped together
  std::vector<int> inv(count, 0);
  int ninv = 0;
  for (int i = 0; i < count; i++) {
    inv[i] = (inst[i].method & 0xff) == HK_INVERSE;
    ninv += inv[i];
    x[i] = MP();
    if (inv[i] && inst[i].shift_hint && !shift_fixed(*inst[i].shift_hint, bt.mats[i]->P.K, x[i]))
      st = dfail_b(HK_EINVAL, "instance " + std::to_string(i) + ": shift hint has more than K fractional bits");
  }
  std::vector<int> solves(count, 0);
  if (ninv > 0 && st == HK_OK) {
    std::vector<int> ok(count, 0), halv(count, 0), a2 = inv;
    for (int attempt = 0; attempt < 5 && st == HK_OK; attempt++) {
      st = factor_batch(bt, x, a2, s, ev, false);
      bool again = false;
      for (int i = 0; i < count && st == HK_OK; i++) {
        if (!a2[i]) continue;
        nfact[i]++;
        const bool above = ev[i].st == HK_ENOTSPD || (ev[i].st == HK_OK && ev[i].first_bad >= 0);
        if (above && !x[i].is_zero()) {
          x[i] = halv[i] < 3 ? shr_mag(x[i], 1) : MP();
          halv[i]++;
          again = true;
        } else {
          a2[i] = 0;
          ok[i] = !above && ev[i].st == HK_OK;
          if (!ok[i]) out[i].status = above ? HK_ENOTSPD : ev[i].st;
        }
      }
      if (!again) break;
    }
    std::vector<MP> li;
    std::vector<hk_status> ist;
    std::vector<int> iters;
    double ts = 0;
    if (st == HK_OK) st = batch_inverse(bt, x, ok, digits, 400, s, li, ist, iters, ts);
    for (int i = 0; i < count && st == HK_OK; i++) {
      if (!ok[i]) continue;
      solves[i] = iters[i];
      if (ist[i] == HK_OK) { lam[i] = li[i]; done[i] = 1; }
      else out[i].status = ist[i];
    }
  }
  // the inertia bracket of "Interval Verification" for every converged instance
  std::vector<MP> xlo(count), xhi(count);
  std::vector<std::string> dec(count);
  for (int i = 0; i < count && st == HK_OK; i++)
    if (done[i]) decimal_bracket(lam[i], bt.mats[i]->P.K, digits, xlo[i], xhi[i], dec[i]);
  std::vector<BEval> elo, ehi;
  bool anydone = false;
  for (int i = 0; i < count; i++) anydone |= done[i] != 0;
  if (paired && anydone && st == HK_OK) {
    // both ends of every bracket in one factorisation
    std::vector<MP> x2(2 * count);
    std::vector<int> a2(2 * count, 0);
    for (int i = 0; i < count; i++)
      if (done[i]) { x2[i] = xlo[i]; x2[count + i] = xhi[i]; a2[i] = a2[count + i] = 1; }
    st = factor_batch(tw, x2, a2, s, ev, false);
    if (st == HK_OK) {
      elo.assign(ev.begin(), ev.begin() + count);
      ehi.assign(ev.begin() + count, ev.end());
    }
  } else {
    if (st == HK_OK) st = factor_batch(bt, xlo, done, s, elo, false);
    if (st == HK_OK) st = factor_batch(bt, xhi, done, s, ehi, false);
  }
  hk_status first = st;
  for (int i = 0; i < count; i++) {
    out[i].factorizations = nfact[i] + (done[i] ? 2 : 0);
    out[i].solves = solves[i];
    out[i].bits_used = bt.mats[i]->P.K;
    out[i].path = 0;
    if (st == HK_OK && done[i]) {
      const int N = bt.mats[i]->P.N;
      const bool okb = elo[i].st == HK_OK && elo[i].nneg == 0 && elo[i].first_bad < 0 &&
                       ehi[i].st == HK_OK && ehi[i].nneg == 1 && ehi[i].first_bad == N - 1;
      out[i].verified = okb ? 1 : 0;
      out[i].status = okb ? HK_OK : HK_EVERIFY;
      snprintf(out[i].lambda_dec, sizeof out[i].lambda_dec, "%s", dec[i].c_str());
      lambda_mpf(lam[i], bt.mats[i]->P.K, &out[i].lambda, out[i].lambda_words);
    }
    if (first == HK_OK && out[i].status != HK_OK) first = out[i].status;
    if (sm[i]) secant_delete(sm[i]);
  }
  if (rep) {
    rep->panel = bt.panel;
    rep->graph_launches = bt.graph_launches + tw.graph_launches;
    rep->t_build_s = std::chrono::duration<double>(t1 - t0).count();
    rep->t_factor_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
    rep->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rep->update_launches = bt.n_update + tw.n_update;
    rep->update_ms = bt.update_ms + tw.update_ms;
    rep->bulk_launches = bt.n_bulk + tw.n_bulk;
    rep->bulk_ms = bt.bulk_ms + tw.bulk_ms;
    int maxW = 0;
    for (const Plan* p : bt.B.plans) maxW = std::max(maxW, p->maxW);
    rep->update_engine = lookahead_mode(bt.lookahead, bt.maxN, maxW) != 2 && mma_width(bt.B, bt.panel) > 0 ? 1 : 0;
  }
  if (first != HK_OK && st == HK_OK) g_err = "some instances failed";
  return first;
}

hk_status hk_autotune(const hk_instance* inst, int count, void* dev_ws, size_t ws_bytes,
                      hipStream_t s, const char* cache_path, int* best_panel, int* best_lookahead,
                      int* best_group) {
  if (!inst || count < 1 || !best_panel) return dfail_b(HK_EINVAL, "bad arguments");
  Batch bt;
  hk_status st = build_batch(bt, inst, count, dev_ws, ws_bytes, s);
  if (st != HK_OK) return st;
  std::vector<MP> x(count);
  std::vector<int> act(count, 1);
  std::vector<BEval> ev;
  // one batched factorisation per candidate (captured and warmed up first)
  auto time_one = [&](int b, int la, int ipw, double& ms) -> hk_status {
    bt.panel = b;
    bt.lookahead = la;
    bt.B.ipw = ipw;
    hk_status e = factor_batch(bt, x, act, s, ev, false);
    if (e != HK_OK) return e;
    auto t0 = std::chrono::steady_clock::now();
    e = factor_batch(bt, x, act, s, ev, false);
    ms = 1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return e;
  };
  const int cand[] = {1, 2, 4, 8, 16};
  double best_ms = 1e300;
  int best = 4, best_la = 0, best_ipw = 4;
  for (int la = 0; la <= 2; la++) {
    for (int b : cand) {
      if (la == 2 && b != 1) continue;   // one column per launch: no panels
      // the in-kernel look-ahead holds the update's operands in LDS too:
      // skipped where its launches do not fit
      if (la == 2 && !factor_lds_check(bt.B, 2).empty()) continue;
      double ms = 0;
      st = time_one(b, la, 4, ms);
      if (st != HK_OK) return st;
      if (ms < best_ms) { best_ms = ms; best = b; best_la = la; }
    }
  }
  // the update workgroup size (items per workgroup) for the best schedule
  if (best_la != 2) {
    for (int ipw : {1, 2}) {
      double ms = 0;
      st = time_one(best, best_la, ipw, ms);
      if (st != HK_OK) return st;
      if (ms < best_ms) { best_ms = ms; best_ipw = ipw; }
    }
  }
  // the update engine: the vector units against the matrix cores (where
  // those apply at this panel width)
  int best_mma = bt.B.mma;
  if (best_la != 2 && mma_width(bt.B, best) > 0) {
    bt.B.mma = 0;
    double ms = 0;
    st = time_one(best, best_la, best_ipw, ms);
    if (st != HK_OK) return st;
    if (ms < best_ms) { best_ms = ms; best_mma = 0; }
    bt.B.mma = 1;
  }
  *best_panel = best;
  if (best_lookahead) *best_lookahead = best_la;
  if (best_group) *best_group = best_ipw;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    if (!f) return dfail_b(HK_EINVAL, "cannot write the tuning cache");
    f << tune_key(inst, count) << " | panel=" << best << " la=" << best_la << " ipw=" << best_ipw
      << " mma=" << best_mma << " ms=" << best_ms << "\n";
  }
  return HK_OK;
}

}  // extern "C"

// ---- batch handles: a batch factored at caller-given shifts, its factors
// readable instance by instance ---------------------------------------------
struct hk_batch_s {
  hk::Batch bt;
};

extern "C" {

hk_status hk_batch_create(const hk_instance* inst, int count, void* dev_ws, size_t ws_bytes, hipStream_t s,
                          hk_batch* out) {
  if (!inst || !out || count < 1) return dfail_b(HK_EINVAL, "bad arguments");
  *out = nullptr;
  hk_batch b = new (std::nothrow) hk_batch_s;
  if (!b) return dfail_b(HK_ENOMEM, "host allocation failed");
  hk_status st = build_batch(b->bt, inst, count, dev_ws, ws_bytes, s);
  if (st != HK_OK) { delete b; return st; }
  const Schedule sc = tuned_schedule(inst, count);
  b->bt.panel = sc.panel > 0 ? sc.panel : 4;
  b->bt.lookahead = sc.lookahead;
  if (sc.ipw > 0) b->bt.B.ipw = sc.ipw;
  if (sc.mma >= 0) b->bt.B.mma = sc.mma;
  *out = b;
  return HK_OK;
}

hk_status hk_batch_set_schedule(hk_batch b, int panel, int lookahead, int group) {
  if (!b || panel < 1 || panel > 64 || lookahead < -1 || lookahead > 2 ||
      (group != 0 && group != 1 && group != 2 && group != 4))
    return dfail_b(HK_EINVAL, "panel must be in 1..64, look-ahead in -1..2 and group 0, 1, 2 or 4");
  b->bt.panel = lookahead == 2 ? 1 : panel;
  b->bt.lookahead = lookahead;
  if (group > 0) b->bt.B.ipw = group;
  return HK_OK;
}

hk_status hk_batch_factor(hk_batch b, const hk_mpf* shifts, hipStream_t s, hk_status* status, int* n_negative,
                          int* first_bad_col) {
  if (!b) return dfail_b(HK_EINVAL, "null batch");
  Batch& bt = b->bt;
  std::vector<MP> x(bt.count);
  std::vector<int> act(bt.count, 1);
  for (int i = 0; i < bt.count && shifts; i++)
    if (!shift_fixed(shifts[i], bt.mats[i]->P.K, x[i]))
      return dfail_b(HK_EINVAL, "shift of instance " + std::to_string(i) + " has more than K fractional bits");
  std::vector<BEval> ev;
  hk_status st = factor_batch(bt, x, act, s, ev, false);
  if (st != HK_OK) return st;
  hk_status first = HK_OK;
  for (int i = 0; i < bt.count; i++) {
    // inertia mode: a last pivot <= 0 is reported, not an error
    const hk_status si = ev[i].st;
    if (status) status[i] = si;
    if (n_negative) n_negative[i] = ev[i].nneg;
    if (first_bad_col) first_bad_col[i] = ev[i].first_bad;
    if (first == HK_OK && si != HK_OK) first = si;
  }
  if (first != HK_OK) g_err = "some instances failed";
  return first;
}

hk_matrix hk_batch_instance(hk_batch b, int i) {
  if (!b || i < 0 || i >= b->bt.count) { g_err = "bad instance index"; return nullptr; }
  return b->bt.mats[i];
}

hk_status hk_batch_destroy(hk_batch b) {
  delete b;
  return HK_OK;
}

}  // extern "C"
