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

namespace {
template <class T>
__global__ __launch_bounds__(256) void transpose_blocks_kernel(const CopySeg* segs, const T* src, T* dst) {
  __shared__ T tile[32][33];
  const CopySeg sg = segs[blockIdx.y];
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8 threads
  for (int tc = 0; tc < sg.cols; tc += 32)
    for (int tr = 0; tr < sg.rows; tr += 32) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = tc + ty + 8 * j, r = tr + tx;
        if (r < sg.rows && c < sg.cols) tile[ty + 8 * j][tx] = src[sg.src + r + int64_t(c) * sg.rows];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = tr + ty + 8 * j, c = tc + tx;
        if (r < sg.rows && c < sg.cols) dst[sg.dst + c + int64_t(r) * sg.cols] = tile[tx][ty + 8 * j];
      }
      __syncthreads();
    }
}
}  // namespace

template <class T>
void launch_transpose_blocks(const CopySeg* segs, int count, const T* src, T* dst, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int c = count - c0 < 65535 ? count - c0 : 65535;
    hipLaunchKernelGGL(transpose_blocks_kernel<T>, dim3(1, c), dim3(256), 0, st, segs + c0, src, dst);
  }
}
template void launch_transpose_blocks<double>(const CopySeg*, int, const double*, double*, hipStream_t);
template void launch_transpose_blocks<float>(const CopySeg*, int, const float*, float*, hipStream_t);

}  // namespace h2
