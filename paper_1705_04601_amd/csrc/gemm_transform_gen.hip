// GEMM launches of the sparsification transforms with a generated operand
// (close blocks formed from the points).
#include "gemm_kc.h"

namespace h2 {

template <class T>
void launch_gemm_transform_gen(const GemmLaunch& g, hipStream_t st) {
  const int m = g.amode * 3 + g.bmode;
  if (m == 6) return launch_layout<T, ROLE_TRANSFORM, 2, 0>(g, st);
  if (m == 7) return launch_layout<T, ROLE_TRANSFORM, 2, 1>(g, st);
}
template void launch_gemm_transform_gen<double>(const GemmLaunch&, hipStream_t);
template void launch_gemm_transform_gen<float>(const GemmLaunch&, hipStream_t);

}  // namespace h2
