// GEMM launches of the sparsification transforms with stored operands.
#include "gemm_kc.h"

namespace h2 {

template <class T>
void launch_gemm_transform(const GemmLaunch& g, hipStream_t st) {
  const int m = g.amode * 3 + g.bmode;
  if (m == 0) return launch_layout<T, ROLE_TRANSFORM, 0, 0>(g, st);
  if (m == 3) return launch_layout<T, ROLE_TRANSFORM, 1, 0>(g, st);
}
template void launch_gemm_transform<double>(const GemmLaunch&, hipStream_t);
template void launch_gemm_transform<float>(const GemmLaunch&, hipStream_t);

}  // namespace h2
