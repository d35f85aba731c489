// Block ILU(0) of S (symmetric form L D L^T) and the solve plan.
#pragma once

#include <memory>

#include "sparse.h"

namespace h2 {

// Device work lists of one preconditioner application for a fixed number of
// right-hand sides.
struct SolvePlan {
  i64 nrhs = 0;
  int64_t tune_gen = 0;                  // tuning generation the lists were planned under
  DeviceBuffer zin, zbuf, y, w, rs, colscale, desc;
  void* zin_ptr = nullptr;               // the vectors' addresses: in the buffers above, or in a
  double* rs_ptr = nullptr;              // scratch arena (allocation-free plans)
  bool eager = false;                    // launched one by one instead of as a captured graph
  std::vector<GemmBatch> up, down;       // U^T and V sweeps, per tree level
  std::vector<GemmBatch> fwd, bwd;       // triangular solves, per DAG level
  GemmBatch diag;                        // D^{-1}
  // long chains of the triangular solves cut into parts: parts after the
  // first store partial sums (in `part`), which a reduction per level then
  // subtracts from the target in part order
  DeviceBuffer part, red;
  void* part_ptr = nullptr;
  void* y_ptr = nullptr;                 // the vectors the fwd and bwd levels update
  void* w_ptr = nullptr;
  const SchurReduce* d_red = nullptr;
  std::vector<int> fred_off, fred_cnt, bred_off, bred_cnt;  // per level: range in d_red
  LaunchGraph apply;                     // the whole application, captured once
};

}  // namespace h2

struct h2_factor {
  h2_sparse* sp = nullptr;
  // active block rows (m > 0) by S position; DAG levels of the elimination
  std::vector<h2::i64> rows;                 // S positions with m > 0
  std::vector<int> flev, blev;               // forward / backward level per S position
  int nflev = 0, nblev = 0;
  std::vector<h2::i64> inv_off;              // per S position: offset of D_k^{-1}
  h2::DeviceBuffer dInv, dZ, dP, dFlag, dDesc;
  h2::i64 pcap = 0;                          // elements of the partial-sum buffer dP
  double flops_schur = 0, flops_inv = 0, flops_z = 0;
  h2::i64 split_targets = 0;                 // Schur targets summed in parts
  h2::i64 schur_launches = 0;                // factorisation levels with Schur work
  double flops_cls[3] = {0, 0, 0};           // Schur flops by tile class (kernel)
  h2::i64 launches_cls[3] = {0, 0, 0};       // Schur kernel launches by tile class
  bool schur_tiled = false;                  // S_kj operands read from tiled copies
  // block threshold ILU: per stored block the square of its drop threshold
  // (fill blocks only; empty in the other modes) and the outcome
  std::vector<double> drop_thr2;
  h2::i64 ilut_dropped = 0, ilut_kept = 0;
  // the factored S with every block transposed (same offsets), made for the
  // backward sweep when it fits beside S; empty otherwise
  h2::DeviceBuffer dST;
  bool st_tried = false;
  std::unique_ptr<h2::SolvePlan> solve;
  ~h2_factor();
};
