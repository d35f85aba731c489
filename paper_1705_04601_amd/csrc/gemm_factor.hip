// GEMM launches of the factorisation (products with the pivot inverses).
#include "gemm_kc.h"

namespace h2 {

template <class T>
void launch_gemm_factor(const GemmLaunch& g, hipStream_t st) {
  if (g.amode * 3 + g.bmode == 0) return launch_layout<T, ROLE_FACTOR, 0, 0>(g, st);
}
template void launch_gemm_factor<double>(const GemmLaunch&, hipStream_t);
template void launch_gemm_factor<float>(const GemmLaunch&, hipStream_t);

}  // namespace h2
