// Sparsified form A = U S U^T of an H^2 matrix (U = V: symmetric kernel).
#pragma once

#include <unordered_map>

#include "batch.h"
#include "h2_internal.h"

namespace h2 {

struct QrLevel {
  std::vector<QrItem> items;       // host copy until uploaded
  const QrItem* d_items = nullptr;
  int count = 0;
  i64 q_begin = 0, q_end = 0;      // range of the level's Q blocks in the Q arena
  i64 w_begin = 0, w_end = 0;      // range of the level's W blocks (coupling factors)
};

struct SweepLevel {
  QrLevel qr;
  GemmBatch stack;                 // R^_c T_c -> B of the father (FP64)
  GemmBatch wproj;                 // W_t = R^_t P_t (FP64)
  GemmBatch strips;                // G Q_p -> S block and carry
  std::vector<GemmBatch> close1, close2;  // chunks: C Q_s, then Q_t^T (.)
  std::vector<GemmBatch> coup1, coup2;    // chunks: K W_b^T, then W_a (.)
  i64 gnext_entries = 0;           // entries of the next level's strip arena to clear
  int gnext_side = 0;              // which of the two strip arenas is "next"
  int nbatches = 0;                // GEMM batches of this level and the ones below (plan)
};

struct PlanCounts {
  double flops_qr = 0, flops_close = 0, flops_coup = 0, flops_strip = 0, flops_misc = 0;
  double bytes_qr = 0;
};

}  // namespace h2

struct h2_sparse {
  h2_matrix* H = nullptr;
  int precision = H2_FP64;
  h2::i64 ncl = 0;
  std::vector<h2::i64> n_act, kept, nonbasis, soff, spos, order;
  // elimination order of the factorisation: levels from the leaves up, inside
  // a level (greedy colour, cluster); S is stored as its upper block triangle
  // in this order (block (t, s) kept with epos(t) <= epos(s))
  std::vector<h2::i64> eorder, epos;
  std::vector<int> colour;
  std::vector<h2::i64> rowptr;     // by elimination position
  std::vector<h2::i64> colidx;     // cluster ids (sorted by elimination position)
  std::vector<h2::i64> blk_off;    // entry offset of each stored block
  h2::i64 s_entries = 0;
  std::vector<char> is_fill;       // per stored block: fill of the exact mode (empty before)
  h2::i64 q_entries = 0;           // entries of the explicit Q_t (symbolic plans)
  bool factored = false;           // S has been overwritten by its factors
  // arenas
  std::vector<h2::i64> q_off, b_off, rhat_off, w_off;
  h2::DeviceBuffer dQ, dQt, dB, dRhat, dW, dWt, dS, dC[2], dG[2], dTmp, dDesc;
  // work lists of the levels above the leaves, uploaded by the sweep while the
  // leaf level runs (plan() uploads the leaf level's only)
  h2::DeviceBuffer dDesc2;
  bool upload_rest = false;
  std::vector<h2::SweepLevel> levels;
  h2::PlanCounts counts;
  size_t elem = 8;                 // bytes per S / transform element
  // Block number of stored block (t, s), or -1: binary search in row epos[t]
  // (columns sorted by elimination position).
  h2::i64 block_of(h2::i64 t, h2::i64 s) const {
    const h2::i64 ps = epos[s];
    h2::i64 lo = rowptr[epos[t]], hi = rowptr[epos[t] + 1];
    while (lo < hi) {
      const h2::i64 mid = (lo + hi) / 2;
      if (epos[colidx[mid]] < ps) lo = mid + 1;
      else hi = mid;
    }
    return (lo < rowptr[epos[t] + 1] && colidx[lo] == s) ? lo : -1;
  }
};

namespace h2 {
void run_sparsify(h2_sparse& sp, hipStream_t st, double* phase_ms);
h2_sparse* plan_sparsify(h2_matrix* H, int precision, bool upload);
h2_sparse* plan_symbolic(h2_matrix* H);
void run_sparsify_batch(std::vector<h2_sparse*>& sps, hipStream_t st, double* phase_ms);
}
