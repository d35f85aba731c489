// GEMM launches of the FP64 H^2 matrix-vector product.
#include "gemm_kc.h"

namespace h2 {

void launch_gemm_matvec(const GemmLaunch& g, hipStream_t st) {
  const int m = g.amode * 3 + g.bmode;
  if (m == 3) return launch_layout<double, ROLE_MATVEC, 1, 0>(g, st);
  if (m == 4) return launch_layout<double, ROLE_MATVEC, 1, 1>(g, st);
  if (m == 5) return launch_layout<double, ROLE_MATVEC, 1, 2>(g, st);
}

}  // namespace h2
