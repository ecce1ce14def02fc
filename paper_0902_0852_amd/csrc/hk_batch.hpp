// The batch object shared by the batched drivers: every instance's workspace
// inside one caller buffer, the device descriptor array, per-instance status
// flags and pivot rows, and the captured graph of one factorisation.
#pragma once
#include <string>
#include <vector>

#include "hk_internal.hpp"

namespace hk {

struct Batch {
  int count = 0, maxN = 0, ld = 0, panel = 4;
  int lookahead = -1, captured_la = -1;   // -1: chosen by size
  std::vector<hk_matrix> mats;
  int borrowed = 0;   // mats[0, borrowed) belong to another batch (a paired batch)
  std::vector<InstDesc> hdesc;
  InstDesc* ddesc = nullptr;
  int32_t* flags = nullptr;
  int32_t* piv = nullptr;
  SweepArgs* sargs = nullptr;   // per-instance solve arguments (batched inverse iteration)
  BatchView B;
  hipStream_t cap = nullptr, cap2 = nullptr;   // capture streams (critical path, look-ahead)
  std::vector<hipEvent_t> events;              // fork/join points of the captured graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int captured_panel = 0, captured_ipw = 0, captured_mma = -1;
  int graph_launches = 0;
  // per-launch timing of the update launches (HK_FLAG_TIME_UPDATES): every
  // factorisation launched one by one on the caller's stream (and s2)
  bool timing = false;
  hipStream_t s2 = nullptr;
  std::vector<hipEvent_t> tevents;
  int n_update = 0, n_bulk = 0;
  double update_ms = 0, bulk_ms = 0;
  Batch() = default;
  Batch(const Batch&) = delete;
  Batch& operator=(const Batch&) = delete;
  ~Batch();
};

// outcome of one instance in a batched factorisation
struct BEval { hk_status st; int nneg, first_bad; std::vector<MP> piv; };

// Lays the batch out in ws (moments on the host, then uploads).
hk_status build_batch(Batch& bt, const hk_instance* inst, int count, void* ws, size_t ws_bytes,
                      hipStream_t s);
// The paired batch of bt: 2 count instances, bt's own (borrowed) and a second
// copy of each with its own workspace in ws (twin_bytes(inst, count) bytes),
// so that two shifts of every instance are factored by one launch sequence.
hk_status build_twin(Batch& tw, Batch& bt, const hk_instance* inst, int count, void* ws, size_t ws_bytes,
                     hipStream_t s);
size_t twin_bytes(const hk_instance* inst, int count);
// One batched factorisation: instance i at shift x[i] (K_i fractional bits)
// when act[i] != 0, replayed from the captured graph; synchronises s.
hk_status factor_batch(Batch& bt, const std::vector<MP>& x, const std::vector<int>& act, hipStream_t s,
                       std::vector<BEval>& out, bool want_pivots);
// bytes of the batch layout (0 and g_err set if an instance is invalid)
size_t batch_bytes(const hk_instance* inst, int count);

// shared with the single-instance drivers (hk_drivers.cpp)
void decimal_bracket(const MP& lam, int K, int digits, MP& xlo, MP& xhi, std::string& dec);
bool parse_decimal(const char* s, int digits, MP& D, int64_t& e);
MP decimal_to_fixed(const MP& D, int64_t e, int K, bool ceil_mode);
std::string decimal_string(const MP& lam, int K, int digits);
// lambda with K fractional bits as an hk_mpf whose digits are words
// (HK_LAMBDA_WORDS of them), rounded to nearest even beyond that
void lambda_mpf(const MP& lam, int K, hk_mpf* out, uint32_t* words);
// |a - b| <= 10^-tol |b| for values with the same number of fractional bits
bool agree(const MP& a, const MP& b, int tol);
// Inverse iteration of every active instance of bt on its current
// factorisation (taken at sigma[i], K_i fractional bits), all instances
// stepped together (hk_binverse.cpp); lam[i] gets K_i fractional bits,
// st[i] the instance's outcome, iters[i] its solves.
hk_status batch_inverse(Batch& bt, const std::vector<MP>& sigma, const std::vector<int>& act, int tol,
                        int max_iter, hipStream_t s, std::vector<MP>& lam, std::vector<hk_status>& st,
                        std::vector<int>& iters, double& t_solve);
// inverse iteration on the current factorisation of m, which was taken at
// shift sigma (K fractional bits); lam gets K fractional bits
hk_status inverse_iterate(hk_matrix m, hipStream_t s, const MP& sigma, int tol, int max_iter, MP& lam,
                          int& solves, double& t_solve);

}  // namespace hk
