// GEMM launches of the solve sweeps (U^T, the triangular solves by DAG
// level, the pivot inverses and V).
#include "gemm_kc.h"

namespace h2 {

template <class T>
void launch_gemm_solve(const GemmLaunch& g, hipStream_t st) {
  const int m = g.amode * 3 + g.bmode;
  if (m == 3) return launch_layout<T, ROLE_SOLVE, 1, 0>(g, st);
  if (m == 4) return launch_layout<T, ROLE_SOLVE, 1, 1>(g, st);
}
template void launch_gemm_solve<double>(const GemmLaunch&, hipStream_t);
template void launch_gemm_solve<float>(const GemmLaunch&, hipStream_t);

}  // namespace h2
