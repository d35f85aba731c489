// HIP kernels of libh2sp for gfx950 (CDNA4, 64-wide wavefronts).
//
//  * gemm_kernel: batched, segmented small GEMM on MFMA (v_mfma_f64_16x16x4 /
//    v_mfma_f32_16x16x4).  One wavefront per 32 x 32 output tile, K staged
//    through LDS in chunks of 16; operand A can be generated on the fly from
//    points (kernel evaluation, so close blocks never touch HBM); the epilogue
//    scatters the four quadrants of the tile to separate destinations (the
//    basis / non-basis split of Section 2).
//  * qr_kernel: Householder QR of a cluster basis held in LDS, FP64, norms by
//    wavefront reductions, explicit square Q (Section 4.2).
//  * inverse_kernel: FP64 Gauss-Jordan inversion with partial pivoting of a
//    pivot block of S, LDS resident.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace h2 {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <class T> struct Mfma;
// Output layout of the 16x16x4 instructions (lane l, accumulator element v):
// f64 holds D[l/16 + 4v][l%16], f32 holds D[4(l/16) + v][l%16] (measured on
// gfx950).  `row` returns that D row.
template <> struct Mfma<double> {
  using V = d4;
  static __device__ __forceinline__ V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return lane / 16 + 4 * v; }
};
template <> struct Mfma<float> {
  using V = f4;
  static __device__ __forceinline__ V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane / 16) + v; }
};

constexpr int TM = 32, TN = 32, KC = 16;

// Destination q of an item, selected with constant indices only (a dynamic
// index into the item's arrays would move the item to scratch memory).
template <class T>
__device__ __forceinline__ void store_out(const GemmItem& it, int q, int lr, int lc, T v, int mode) {
  void* b;
  int64_t ld;
  bool tr;
  switch (q) {
    case 0: b = it.out[0]; ld = it.ld[0]; tr = it.trans[0]; break;
    case 1: b = it.out[1]; ld = it.ld[1]; tr = it.trans[1]; break;
    case 2: b = it.out[2]; ld = it.ld[2]; tr = it.trans[2]; break;
    case 3: b = it.out[3]; ld = it.ld[3]; tr = it.trans[3]; break;
    default: b = it.out[4]; ld = it.ld[4]; tr = it.trans[4]; break;
  }
  T* base = static_cast<T*>(b);
  if (!base) return;
  T* p = tr ? base + lc + lr * ld : base + lr + lc * ld;
  if (mode == GEMM_STORE) *p = v;
  else if (mode == GEMM_ADD) *p += v;
  else *p -= v;
}

template <class T, int ROLE>
__global__ __launch_bounds__(64) void gemm_kernel(GemmLaunch g) {
  using V = typename Mfma<T>::V;
  __shared__ T As[KC][TM + 1];
  __shared__ T Bs[KC][TN + 1];
  const int lane = threadIdx.x;
  const uint32_t code = static_cast<uint32_t>(g.tiles[blockIdx.x]);
  const GemmItem it = g.items[code >> 8];
  const int m0 = int((code >> 4) & 15) * TM, n0 = int(code & 15) * TN;
  V acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = V{0, 0, 0, 0};
  const int dim = it.gdim;
  for (int si = it.seg_begin; si < it.seg_end; ++si) {
    const GemmSeg sg = g.segs[si];
    for (int k0 = 0; k0 < sg.K; k0 += KC) {
      // ---- A chunk (TM x KC) into As[k][m]
      if (sg.gen) {
        const double* pr = static_cast<const double*>(sg.A);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int idx = lane + 64 * e, i = idx % TM, k = idx / TM;
          const int gi = m0 + i, gk = k0 + k;
          T v = T(0);
          if (gi < it.M && gk < sg.K) {
            if (sg.diag && gi == gk) {
              v = T(it.gdiag);
            } else {
              double d2 = 0.0;
              for (int a = 0; a < dim; ++a) {
                const double d = pr[gi * dim + a] - sg.pc[gk * dim + a];
                d2 += d * d;
              }
              v = T(it.gscale / sqrt(d2));
            }
          }
          As[k][i] = v;
        }
      } else if (sg.opA == 0) {
        const T* A = static_cast<const T*>(sg.A);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int idx = lane + 64 * e, i = idx % TM, k = idx / TM;
          const int gi = m0 + i, gk = k0 + k;
          As[k][i] = (gi < it.M && gk < sg.K) ? A[gi + int64_t(gk) * sg.lda] : T(0);
        }
      } else {
        const T* A = static_cast<const T*>(sg.A);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int idx = lane + 64 * e, k = idx % KC, i = idx / KC;
          const int gi = m0 + i, gk = k0 + k;
          As[k][i] = (gi < it.M && gk < sg.K) ? A[gk + int64_t(gi) * sg.lda] : T(0);
        }
      }
      // ---- B chunk (KC x TN) into Bs[k][n]
      const T* B = static_cast<const T*>(sg.B);
      if (sg.opB == 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int idx = lane + 64 * e, k = idx % KC, n = idx / KC;
          const int gk = k0 + k, gn = n0 + n;
          Bs[k][n] = (gk < sg.K && gn < it.N) ? B[gk + int64_t(gn) * sg.ldb] : T(0);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int idx = lane + 64 * e, n = idx % TN, k = idx / TN;
          const int gk = k0 + k, gn = n0 + n;
          Bs[k][n] = (gk < sg.K && gn < it.N) ? B[gn + int64_t(gk) * sg.ldb] : T(0);
        }
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const int kr = kk + lane / 16, c = lane % 16;
        const T a0 = As[kr][c], a1 = As[kr][16 + c];
        const T b0 = Bs[kr][c], b1 = Bs[kr][16 + c];
        // operands swapped (D = B^T A^T) so that consecutive lanes hold
        // consecutive output rows: lane l has output row 16bm + l%16 and
        // output column 16bn + Mfma<T>::row(l, v)
        acc[0][0] = Mfma<T>::run(b0, a0, acc[0][0]);
        acc[0][1] = Mfma<T>::run(b1, a0, acc[0][1]);
        acc[1][0] = Mfma<T>::run(b0, a1, acc[1][0]);
        acc[1][1] = Mfma<T>::run(b1, a1, acc[1][1]);
      }
      __syncthreads();
    }
  }
  // ---- epilogue: quadrant scatter
  for (int bm = 0; bm < 2; ++bm)
    for (int bn = 0; bn < 2; ++bn)
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + 16 * bm + lane % 16;
        const int col = n0 + 16 * bn + Mfma<T>::row(lane, v);
        if (row >= it.M || col >= it.N) continue;
        const int q = (row >= it.rs ? 2 : 0) + (col >= it.cs ? 1 : 0);
        const int lr = row - (q >= 2 ? it.rs : 0), lc = col - ((q & 1) ? it.cs : 0);
        const T val = acc[bm][bn][v];
        store_out<T>(it, q, lr, lc, val, g.mode);
        if (q == 0) store_out<T>(it, 4, lr, lc, val, g.mode);
      }
}

// K-contiguous variant: A stored K x M (op(A) = A^T) and B stored K x N, so
// both operands run along K in memory.  No LDS: lane l loads 4 consecutive k
// (k0 + 4(l/16) .. +3) of its row of A and of its column of B and feeds them
// to 4 consecutive MFMAs.  Inside one instruction the four lane groups then
// carry k = k0 + 4g + s (g = 0..3) for step s: A and B agree on that
// permutation of K, and the four steps cover all 16 values of k.  A wave owns
// a tile of up to 4 x 4 MFMA blocks (64 x 64), sized to the item so that
// blocks of 48 or 16 rows waste no lanes.
template <class T> struct Vec4;
template <> struct Vec4<float> { typedef float type __attribute__((ext_vector_type(4), aligned(4))); };
template <> struct Vec4<double> { typedef double type __attribute__((ext_vector_type(4), aligned(8))); };

template <class T>
__device__ __forceinline__ void load4(const T* p, int k, int K, bool ok, T* v) {
  if (ok && k + 3 < K) {
    const typename Vec4<T>::type x = *reinterpret_cast<const typename Vec4<T>::type*>(p + k);
    v[0] = x[0];
    v[1] = x[1];
    v[2] = x[2];
    v[3] = x[3];
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = (ok && k + s < K) ? p[k + s] : T(0);
  }
}

constexpr int KT = 64;  // tile edge of the K-contiguous kernels

// Work-groups are handed to the 8 XCDs round-robin by block index, and each
// XCD has its own L2.  Tile lists put tiles that share operands next to each
// other; this mapping gives XCD x the x-th contiguous eighth of the list, so
// neighbouring tiles meet in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int x = b % 8, q = b / 8, base = n / 8, rem = n % 8;
  return x * base + min(x, rem) + q;
}

// Operand fetch of the direct kernel for one 16-row (or 16-column) block and
// the four k of this lane: K-contiguous rows (vector load), M-contiguous
// columns (one load per k, coalesced across the 16 lanes of a group) or
// generated kernel values.
template <class T, int MODE>
__device__ __forceinline__ void fetch4(const T* p, int64_t ld, int row, int k, int K, bool ok, T* v,
                                       const double* pr, const double* pc, int dim, double scale, double dg,
                                       bool diag) {
  if (MODE == 0) {          // element (row, k) at p[k + row ld]
    load4<T>(p, k, K, ok, v);
  } else if (MODE == 1) {   // element (row, k) at p[row + k ld]
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = (ok && k + s < K) ? p[row + int64_t(k + s) * ld] : T(0);
  } else {                  // generated: scale / |pr_row - pc_k|, dg on the diagonal
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      T val = T(0);
      if (ok && k + s < K) {
        if (diag && row == k + s) {
          val = T(dg);
        } else {
          double d2 = 0.0;
          for (int a = 0; a < dim; ++a) {
            const double d = pr[row * dim + a] - pc[(k + s) * dim + a];
            d2 += d * d;
          }
          val = T(scale / sqrt(d2));
        }
      }
      v[s] = val;
    }
  }
}

// acc += op(A) op(B) for one segment; AM / BM select the fetch of each operand.
template <class T, int AM, int BM>
__device__ __forceinline__ void direct_segment(typename Mfma<T>::V (&acc)[4][4], int nbm, int nbn,
                                               const GemmSeg& sg, int m0, int n0, int M, int N, int lane,
                                               int dim, double scale, double dg) {
  const int r = lane % 16, kq = 4 * (lane / 16);
  const T* A = static_cast<const T*>(sg.A);
  const T* B = static_cast<const T*>(sg.B);
  const double* pr = static_cast<const double*>(sg.A);
  const int K = sg.K;
  const T* pa[4];
  const T* pb[4];
  int ra[4], cb[4];
  bool oa[4], ob[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    ra[b] = m0 + 16 * b + r;
    cb[b] = n0 + 16 * b + r;
    oa[b] = b < nbm && ra[b] < M;
    ob[b] = b < nbn && cb[b] < N;
    pa[b] = (AM == 0) ? A + int64_t(oa[b] ? ra[b] : 0) * sg.lda : A;
    pb[b] = (BM == 0) ? B + int64_t(ob[b] ? cb[b] : 0) * sg.ldb : B;
  }
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int k = k0 + kq;
    T a[4][4], bv[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b < nbm) fetch4<T, AM>(pa[b], sg.lda, ra[b], k, K, oa[b], a[b], pr, sg.pc, dim, scale, dg, sg.diag);
      if (b < nbn) fetch4<T, BM>(pb[b], sg.ldb, cb[b], k, K, ob[b], bv[b], nullptr, nullptr, 0, 0.0, 0.0, false);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int bm = 0; bm < 4; ++bm)
#pragma unroll
        for (int bn = 0; bn < 4; ++bn)
          if (bm < nbm && bn < nbn) acc[bm][bn] = Mfma<T>::run(bv[bn][s], a[bm][s], acc[bm][bn]);
  }
}

template <class T, int ROLE>
__global__ __launch_bounds__(64) void gemm_kc_kernel(GemmLaunch g) {
  using V = typename Mfma<T>::V;
  const int lane = threadIdx.x;
  // the solve and matvec lists interleave heavy and light items: keep their
  // round-robin spread over the XCDs
  const int tb = (ROLE == ROLE_TRANSFORM || ROLE == ROLE_FACTOR) ? xcd_tile(blockIdx.x, gridDim.x) : int(blockIdx.x);
  const uint32_t code = static_cast<uint32_t>(g.tiles[tb]);
  const GemmItem it = g.items[code >> 8];
  const int m0 = int((code >> 4) & 15) * KT, n0 = int(code & 15) * KT;
  const int nbm = min(4, (it.M - m0 + 15) / 16), nbn = min(4, (it.N - n0 + 15) / 16);
  V acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = V{0, 0, 0, 0};
  for (int si = it.seg_begin; si < it.seg_end; ++si) {
    const GemmSeg sg = g.segs[si];
    // operand layouts: A K-contiguous (opA = 1), M-contiguous (opA = 0) or
    // generated; B K-contiguous (opB = 0) or N-contiguous (opB = 1)
    const int am = sg.gen ? 2 : (sg.opA ? 0 : 1);
    const int bmode = sg.opB ? 1 : 0;
    if (am == 0 && bmode == 0)
      direct_segment<T, 0, 0>(acc, nbm, nbn, sg, m0, n0, it.M, it.N, lane, it.gdim, it.gscale, it.gdiag);
    else if (am == 1 && bmode == 0)
      direct_segment<T, 1, 0>(acc, nbm, nbn, sg, m0, n0, it.M, it.N, lane, it.gdim, it.gscale, it.gdiag);
    else if (am == 2 && bmode == 0)
      direct_segment<T, 2, 0>(acc, nbm, nbn, sg, m0, n0, it.M, it.N, lane, it.gdim, it.gscale, it.gdiag);
    else if (am == 0)
      direct_segment<T, 0, 1>(acc, nbm, nbn, sg, m0, n0, it.M, it.N, lane, it.gdim, it.gscale, it.gdiag);
    else if (am == 1)
      direct_segment<T, 1, 1>(acc, nbm, nbn, sg, m0, n0, it.M, it.N, lane, it.gdim, it.gscale, it.gdiag);
    else
      direct_segment<T, 2, 1>(acc, nbm, nbn, sg, m0, n0, it.M, it.N, lane, it.gdim, it.gscale, it.gdiag);
  }
#pragma unroll
  for (int bm = 0; bm < 4; ++bm)
#pragma unroll
    for (int bn = 0; bn < 4; ++bn) {
      if (bm >= nbm || bn >= nbn) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + 16 * bm + lane % 16;
        const int col = n0 + 16 * bn + Mfma<T>::row(lane, v);
        if (row >= it.M || col >= it.N) continue;
        const int q = (row >= it.rs ? 2 : 0) + (col >= it.cs ? 1 : 0);
        const int lr = row - (q >= 2 ? it.rs : 0), lc = col - ((q & 1) ? it.cs : 0);
        const T val = acc[bm][bn][v];
        store_out<T>(it, q, lr, lc, val, g.mode);
        if (q == 0) store_out<T>(it, 4, lr, lc, val, g.mode);
      }
    }
}

// Schur update of the block factorisation with compact descriptors:
// S[out] (M x N, ld M) -= sum_seg Z[a]^T (K x M, ld K) S[b] (K x N, ld K).
// One wave per 64 x 64 tile.  The (segment, 16-wide k step) pairs form one
// chunk stream, consumed with two register sets in ping-pong: the loads of
// chunk c + 1 are in flight while the MFMAs of chunk c issue.  The number of
// 16 x 16 blocks of the tile (NBM x NBN) is a template parameter and every
// load is issued unconditionally, so the count of loads in flight is static
// and the compiler waits only for the older set.  Z_ki is stored with its K
// rounded up to 16 and zero rows below K, so a chunk may run past the end of
// a segment: the extra k multiply zeros of Z by finite entries of S (the
// over-read stays inside S, which is allocated with kOverread zeroed spare
// elements at its end).
template <class T, int NBM, int NBN>
__device__ __forceinline__ void schur_fetch(const T* S, const T* Z, const SchurSeg& sg, int k0, bool valid,
                                            const T* zeros, int m0, int n0, int M, int N, int r, int kq,
                                            T (&a)[4][4], T (&b)[4][4]) {
  // no arithmetic on the loaded values (it would make the wave wait for them
  // at once): rows past the tile read a valid row and land in discarded
  // outputs; k past the segment meets the zero rows of the padded Z_ki; a
  // chunk past the item's end reads zeros
  const int k = k0 + kq, lda = (sg.K + 15) & ~15;
#pragma unroll
  for (int q = 0; q < NBM; ++q) {
    const int row = m0 + 16 * q + r;
    const T* p = valid ? Z + sg.a_off + int64_t(row < M ? row : 0) * lda + k : zeros;
    const typename Vec4<T>::type x = *reinterpret_cast<const typename Vec4<T>::type*>(p);
#pragma unroll
    for (int s = 0; s < 4; ++s) a[q][s] = x[s];
  }
#pragma unroll
  for (int q = 0; q < NBN; ++q) {
    const int col = n0 + 16 * q + r;
    const T* p = valid ? S + sg.b_off + int64_t(col < N ? col : 0) * sg.K + k : zeros;
    const typename Vec4<T>::type x = *reinterpret_cast<const typename Vec4<T>::type*>(p);
#pragma unroll
    for (int s = 0; s < 4; ++s) b[q][s] = x[s];
  }
}

template <class T, int NBM, int NBN>
__device__ __forceinline__ void schur_mfma(typename Mfma<T>::V (&acc)[4][4], const T (&a)[4][4], const T (&b)[4][4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int bm = 0; bm < NBM; ++bm)
#pragma unroll
      for (int bn = 0; bn < NBN; ++bn) acc[bm][bn] = Mfma<T>::run(b[bn][s], a[bm][s], acc[bm][bn]);
}

// Chunk cursor: segment index, first k of the chunk, the segment; valid is
// false past the item's last segment (and stays false).
struct SchurCursor {
  int si, k0;
  bool valid;
  SchurSeg sg;
};

__device__ __forceinline__ SchurCursor schur_next(const SchurSeg* segs, int seg_end, SchurCursor c) {
  if (!c.valid) return c;
  c.k0 += 16;
  if (c.k0 < c.sg.K) return c;
  ++c.si;
  c.k0 = 0;
  if (c.si >= seg_end) {
    c.valid = false;
    return c;
  }
  c.sg = segs[c.si];
  return c;
}

template <class T, int NBM, int NBN>
__device__ __forceinline__ void schur_tile(const SchurLaunch& g, const SchurItem& it, int m0, int n0, int lane) {
  using V = typename Mfma<T>::V;
  const int r = lane % 16, kq = 4 * (lane / 16);
  T* S = static_cast<T*>(g.S);
  const T* Z = static_cast<const T*>(g.Z);
  const T* zeros = static_cast<const T*>(g.zeros);
  V acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = V{0, 0, 0, 0};
  if (it.seg_begin < it.seg_end) {
    T a0[4][4], b0[4][4], a1[4][4], b1[4][4];
    SchurCursor c{it.seg_begin, 0, true, g.segs[it.seg_begin]};
    schur_fetch<T, NBM, NBN>(S, Z, c.sg, c.k0, true, zeros, m0, n0, it.M, it.N, r, kq, a0, b0);
    // two chunks per pass, one exit: the second chunk of the last pass may
    // be past the end and then contributes zeros
    while (true) {
      const SchurCursor c1 = schur_next(g.segs, it.seg_end, c);
      schur_fetch<T, NBM, NBN>(S, Z, c1.sg, c1.k0, c1.valid, zeros, m0, n0, it.M, it.N, r, kq, a1, b1);
      schur_mfma<T, NBM, NBN>(acc, a0, b0);
      const SchurCursor c2 = schur_next(g.segs, it.seg_end, c1);
      schur_fetch<T, NBM, NBN>(S, Z, c2.sg, c2.k0, c2.valid, zeros, m0, n0, it.M, it.N, r, kq, a0, b0);
      schur_mfma<T, NBM, NBN>(acc, a1, b1);
      if (!c2.valid) break;
      c = c2;
    }
  }
  const bool part = it.partial != 0;
  T* out = (part ? static_cast<T*>(g.P) : S) + it.out_off;
#pragma unroll
  for (int bm = 0; bm < NBM; ++bm)
#pragma unroll
    for (int bn = 0; bn < NBN; ++bn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + 16 * bm + r;
        const int col = n0 + 16 * bn + Mfma<T>::row(lane, v);
        if (row < it.M && col < it.N) {
          T* o = out + row + int64_t(col) * it.M;
          if (part) *o = acc[bm][bn][v];
          else *o -= acc[bm][bn][v];
        }
      }
}

template <class T>
__global__ __launch_bounds__(64) void schur_kernel(SchurLaunch g) {
  const int lane = threadIdx.x;
  const uint32_t code = static_cast<uint32_t>(g.tiles[xcd_tile(blockIdx.x, gridDim.x)]);
  const SchurItem it = g.items[code >> 8];
  const int m0 = int((code >> 4) & 15) * KT, n0 = int(code & 15) * KT;
  const int nbm = min(4, (it.M - m0 + 15) / 16), nbn = min(4, (it.N - n0 + 15) / 16);
  switch (nbm * 4 + nbn) {
#define H2_SCHUR_CASE(I, J) \
  case I * 4 + J: schur_tile<T, I, J>(g, it, m0, n0, lane); break;
    H2_SCHUR_CASE(1, 1) H2_SCHUR_CASE(1, 2) H2_SCHUR_CASE(1, 3) H2_SCHUR_CASE(1, 4)
    H2_SCHUR_CASE(2, 1) H2_SCHUR_CASE(2, 2) H2_SCHUR_CASE(2, 3) H2_SCHUR_CASE(2, 4)
    H2_SCHUR_CASE(3, 1) H2_SCHUR_CASE(3, 2) H2_SCHUR_CASE(3, 3) H2_SCHUR_CASE(3, 4)
    H2_SCHUR_CASE(4, 1) H2_SCHUR_CASE(4, 2) H2_SCHUR_CASE(4, 3) H2_SCHUR_CASE(4, 4)
#undef H2_SCHUR_CASE
    default: break;
  }
}

// S[target] -= sum of the target's partial sums, in part order.
template <class T>
__global__ void schur_reduce_kernel(const SchurReduce* items, const T* P, T* S) {
  const SchurReduce r = items[blockIdx.y];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < r.len; e += gridDim.x * blockDim.x) {
    T acc = T(0);
    for (int p = 0; p < r.parts; ++p) acc += P[r.p_off + int64_t(p) * r.len + e];
    S[r.s_off + e] -= acc;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(256) void qr_kernel(const QrItem* items) {
  __shared__ double Bs[128 * 64];
  __shared__ double Qs[128 * 32];
  __shared__ double tau[64];
  __shared__ double scal[2];
  const QrItem it = items[blockIdx.x];
  const int n = it.n, r = it.r, kk = it.k, tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  if (kk == 0) {
    for (int e = tid; e < n * n; e += 256) it.Q[e] = (e % n == e / n) ? 1.0 : 0.0;
    return;
  }
  for (int e = tid; e < n * r; e += 256) Bs[e] = it.B[e];
  __syncthreads();
  const int q = n < r ? n : r;
  for (int j = 0; j < q; ++j) {
    if (wave == 0) {
      double s = 0.0;
      for (int i = j + 1 + lane; i < n; i += 64) s += Bs[i + j * n] * Bs[i + j * n];
      s = wave_sum(s);
      if (lane == 0) {
        const double alpha = Bs[j + j * n];
        if (s == 0.0) {
          tau[j] = 0.0;
        } else {
          const double nrm = sqrt(alpha * alpha + s);
          const double beta = alpha >= 0.0 ? -nrm : nrm;
          tau[j] = (beta - alpha) / beta;
          scal[0] = 1.0 / (alpha - beta);
          scal[1] = beta;
        }
      }
    }
    __syncthreads();
    const double tj = tau[j];
    if (tj != 0.0) {
      const double sc = scal[0];
      for (int i = j + 1 + tid; i < n; i += 256) Bs[i + j * n] *= sc;
      if (tid == 0) Bs[j + j * n] = scal[1];
      __syncthreads();
      for (int c = j + 1 + wave; c < r; c += 4) {
        double d = 0.0;
        for (int i = j + 1 + lane; i < n; i += 64) d += Bs[i + j * n] * Bs[i + c * n];
        d = wave_sum(d);
        d = (d + Bs[j + c * n]) * tj;
        for (int i = j + 1 + lane; i < n; i += 64) Bs[i + c * n] -= d * Bs[i + j * n];
        if (lane == 0) Bs[j + c * n] -= d;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < kk * r; e += 256) {
    const int i = e % kk, j = e / kk;
    it.Rhat[e] = (i <= j) ? Bs[i + j * n] : 0.0;
  }
  const int cc = tid / 8, sub = tid % 8;
  for (int c0 = 0; c0 < n; c0 += 32) {
    const int nc = (n - c0) < 32 ? (n - c0) : 32;
    for (int e = tid; e < n * 32; e += 256) {
      const int i = e % n, c = e / n;
      Qs[e] = (c < nc && i == c0 + c) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int jtop = (q - 1) < (c0 + 31) ? (q - 1) : (c0 + 31);
    if (cc < nc) {
      for (int j = jtop; j >= 0; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;
        double d = 0.0;
        for (int i = j + 1 + sub; i < n; i += 8) d += Bs[i + j * n] * Qs[i + cc * n];
        d += __shfl_xor(d, 4, 64);
        d += __shfl_xor(d, 2, 64);
        d += __shfl_xor(d, 1, 64);
        d = (d + Qs[j + cc * n]) * tj;
        for (int i = j + 1 + sub; i < n; i += 8) Qs[i + cc * n] -= d * Bs[i + j * n];
        if (sub == 0) Qs[j + cc * n] -= d;
      }
    }
    __syncthreads();
    for (int e = tid; e < n * nc; e += 256) it.Q[int64_t(c0) * n + e] = Qs[e];
    __syncthreads();
  }
}

template <class T>
__global__ __launch_bounds__(256) void inverse_kernel(const InvItem<T>* items, int* flag) {
  __shared__ double a[128 * 128];
  __shared__ double fcol[128];
  __shared__ int perm[128];
  const InvItem<T> it = items[blockIdx.x];
  const int m = it.m, tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  for (int e = tid; e < m * m; e += 256) a[e] = double(it.A[e]);
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    if (wave == 0) {
      double best = -1.0;
      int bi = j;
      for (int i = j + lane; i < m; i += 64) {
        const double v = fabs(a[i + j * m]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        perm[j] = bi;
        if (!(best > 0.0)) atomicOr(flag, 1);
      }
    }
    __syncthreads();
    const int p = perm[j];
    if (p != j)
      for (int c = tid; c < m; c += 256) {
        const double t = a[j + c * m];
        a[j + c * m] = a[p + c * m];
        a[p + c * m] = t;
      }
    __syncthreads();
    const double piv = a[j + j * m];
    for (int i = tid; i < m; i += 256) fcol[i] = a[i + j * m];
    __syncthreads();
    for (int c = tid; c < m; c += 256) a[j + c * m] = (c == j ? 1.0 : a[j + c * m]) / piv;
    __syncthreads();
    for (int e = tid; e < m * m; e += 256) {
      const int i = e % m, c = e / m;
      if (i != j) a[e] = (c == j ? 0.0 : a[e]) - fcol[i] * a[j + c * m];
    }
    __syncthreads();
  }
  for (int j = m - 1; j >= 0; --j) {
    const int p = perm[j];
    if (p != j)
      for (int i = tid; i < m; i += 256) {
        const double t = a[i + j * m];
        a[i + j * m] = a[i + p * m];
        a[i + p * m] = t;
      }
    __syncthreads();
  }
  for (int e = tid; e < m * m; e += 256) it.Inv[e] = T(a[e]);
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}
__global__ void fill_f_kernel(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}
__global__ void fill_i_kernel(int* p, int64_t n, int v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}
__global__ void cast_d2f_kernel(const double* in, float* out, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) out[i] = float(in[i]);
}
__global__ void cast_f2d_kernel(const float* in, double* out, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) out[i] = double(in[i]);
}
template <class T>
__global__ void gather_rows_kernel(const T* in, int64_t ldi, const int64_t* idx, T* out, int64_t ldo, int64_t n, int64_t nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e % n, j = e / n;
    out[i + j * ldo] = in[idx[i] + j * ldi];
  }
}
__global__ void scatter_rows_kernel(const double* in, int64_t ldi, const int64_t* idx, double* out, int64_t ldo, int64_t n, int64_t nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e % n, j = e / n;
    out[idx[i] + j * ldo] = in[i + j * ldi];
  }
}
// one block per column: r = b - y and the sums of squares of r and b
__global__ __launch_bounds__(256) void residual_kernel(const double* b, int64_t ldb, const double* y, int64_t ldy, double* r,
                                                       int64_t n, double* nrm2, int64_t nrhs) {
  __shared__ double red[2][256];
  const int64_t j = blockIdx.x;
  double sr = 0.0, sb = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double bv = b[i + j * ldb];
    const double rv = bv - y[i + j * ldy];
    r[i + j * n] = rv;
    sr += rv * rv;
    sb += bv * bv;
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = sb;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    nrm2[j] = red[0][0];
    nrm2[nrhs + j] = red[1][0];
  }
}
__global__ void scale_to_f_kernel(const double* in, const double* cs, float* out, int64_t n, int64_t nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x)
    out[e] = float(in[e] / cs[e / n]);
}
__global__ void add_scaled_f_kernel(const float* in, const double* cs, double* acc, int64_t ldacc, int64_t n, int64_t nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e % n, j = e / n;
    acc[i + j * ldacc] += double(in[e]) * cs[j];
  }
}
__global__ void add_kernel(const double* in, double* acc, int64_t ldacc, int64_t n, int64_t nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e % n, j = e / n;
    acc[i + j * ldacc] += in[e];
  }
}
__global__ void copy_cols_kernel(const double* in, int64_t ldi, double* out, int64_t ldo, int64_t n, int64_t nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e % n, j = e / n;
    out[i + j * ldo] = in[i + j * ldi];
  }
}

template <class T>
__global__ void copy_segments_kernel(const CopySeg* segs, const T* src, T* dst) {
  const CopySeg s = segs[blockIdx.y];
  const int len = s.rows * s.cols;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < len; e += gridDim.x * blockDim.x) {
    const int c = e / s.rows, r = e - c * s.rows;
    dst[s.dst + e] = src[s.src + int64_t(c) * s.src_ld + r];
  }
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return int(g);
}

}  // namespace

template <class T>
void launch_gemm(const GemmLaunch& g, hipStream_t st) {
  if (g.ntiles <= 0) return;
  if (g.kc) {
    switch (g.role) {
      case ROLE_FACTOR: hipLaunchKernelGGL((gemm_kc_kernel<T, ROLE_FACTOR>), dim3(g.ntiles), dim3(64), 0, st, g); break;
      case ROLE_SOLVE: hipLaunchKernelGGL((gemm_kc_kernel<T, ROLE_SOLVE>), dim3(g.ntiles), dim3(64), 0, st, g); break;
      case ROLE_MATVEC: hipLaunchKernelGGL((gemm_kc_kernel<T, ROLE_MATVEC>), dim3(g.ntiles), dim3(64), 0, st, g); break;
      default: hipLaunchKernelGGL((gemm_kc_kernel<T, ROLE_TRANSFORM>), dim3(g.ntiles), dim3(64), 0, st, g); break;
    }
    return;
  }
  switch (g.role) {
    case ROLE_FACTOR: hipLaunchKernelGGL((gemm_kernel<T, ROLE_FACTOR>), dim3(g.ntiles), dim3(64), 0, st, g); break;
    case ROLE_SOLVE: hipLaunchKernelGGL((gemm_kernel<T, ROLE_SOLVE>), dim3(g.ntiles), dim3(64), 0, st, g); break;
    case ROLE_MATVEC: hipLaunchKernelGGL((gemm_kernel<T, ROLE_MATVEC>), dim3(g.ntiles), dim3(64), 0, st, g); break;
    default: hipLaunchKernelGGL((gemm_kernel<T, ROLE_TRANSFORM>), dim3(g.ntiles), dim3(64), 0, st, g); break;
  }
}
template void launch_gemm<double>(const GemmLaunch&, hipStream_t);
template void launch_gemm<float>(const GemmLaunch&, hipStream_t);

template <class T>
void launch_schur(const SchurLaunch& g, hipStream_t st) {
  if (g.ntiles <= 0) return;
  hipLaunchKernelGGL(schur_kernel<T>, dim3(g.ntiles), dim3(64), 0, st, g);
}
template void launch_schur<double>(const SchurLaunch&, hipStream_t);
template void launch_schur<float>(const SchurLaunch&, hipStream_t);

template <class T>
void launch_schur_reduce(const SchurReduce* items, int count, const T* P, T* S, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int c = count - c0 < 65535 ? count - c0 : 65535;
    hipLaunchKernelGGL(schur_reduce_kernel<T>, dim3(16, c), dim3(256), 0, st, items + c0, P, S);
  }
}
template void launch_schur_reduce<double>(const SchurReduce*, int, const double*, double*, hipStream_t);
template void launch_schur_reduce<float>(const SchurReduce*, int, const float*, float*, hipStream_t);

void launch_qr(const QrItem* items, int count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(qr_kernel, dim3(count), dim3(256), 0, st, items);
}

template <class T>
void launch_inverse(const InvItem<T>* items, int count, int* flag, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(inverse_kernel<T>, dim3(count), dim3(256), 0, st, items, flag);
}
template void launch_inverse<double>(const InvItem<double>*, int, int*, hipStream_t);
template void launch_inverse<float>(const InvItem<float>*, int, int*, hipStream_t);

template <class T>
void launch_copy_segments(const CopySeg* segs, int count, const T* src, T* dst, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int c = (count - c0) < 65535 ? (count - c0) : 65535;
    hipLaunchKernelGGL(copy_segments_kernel<T>, dim3(64, c), dim3(256), 0, st, segs + c0, src, dst);
  }
}
template void launch_copy_segments<double>(const CopySeg*, int, const double*, double*, hipStream_t);
template void launch_copy_segments<float>(const CopySeg*, int, const float*, float*, hipStream_t);

void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
}
void launch_fill_f(float* p, int64_t n, float v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(fill_f_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
}
void launch_fill_i(int* p, int64_t n, int v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(fill_i_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
}
void launch_cast_d2f(const double* in, float* out, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(cast_d2f_kernel, dim3(grid_for(n)), dim3(256), 0, st, in, out, n);
}
void launch_cast_f2d(const float* in, double* out, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(cast_f2d_kernel, dim3(grid_for(n)), dim3(256), 0, st, in, out, n);
}
template <class T>
void launch_gather_rows(const T* in, int64_t ldi, const int64_t* idx, T* out, int64_t ldo, int64_t n, int64_t nrhs,
                        hipStream_t st) {
  if (n * nrhs > 0)
    hipLaunchKernelGGL(gather_rows_kernel<T>, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, ldi, idx, out, ldo, n, nrhs);
}
template void launch_gather_rows<double>(const double*, int64_t, const int64_t*, double*, int64_t, int64_t, int64_t, hipStream_t);
void launch_scatter_rows(const double* in, int64_t ldi, const int64_t* idx, double* out, int64_t ldo, int64_t n,
                         int64_t nrhs, hipStream_t st) {
  if (n * nrhs > 0)
    hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, ldi, idx, out, ldo, n, nrhs);
}
void launch_residual(const double* b, int64_t ldb, const double* y, int64_t ldy, double* r, int64_t n, int64_t nrhs,
                     double* nrm2, hipStream_t st) {
  if (nrhs > 0) hipLaunchKernelGGL(residual_kernel, dim3(nrhs), dim3(256), 0, st, b, ldb, y, ldy, r, n, nrm2, nrhs);
}
void launch_scale_to_f(const double* in, const double* cs, float* out, int64_t n, int64_t nrhs, hipStream_t st) {
  if (n * nrhs > 0) hipLaunchKernelGGL(scale_to_f_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, cs, out, n, nrhs);
}
void launch_add_scaled_f(const float* in, const double* cs, double* acc, int64_t ldacc, int64_t n, int64_t nrhs,
                         hipStream_t st) {
  if (n * nrhs > 0)
    hipLaunchKernelGGL(add_scaled_f_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, cs, acc, ldacc, n, nrhs);
}
void launch_add(const double* in, double* acc, int64_t ldacc, int64_t n, int64_t nrhs, hipStream_t st) {
  if (n * nrhs > 0) hipLaunchKernelGGL(add_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, acc, ldacc, n, nrhs);
}
void launch_copy_cols(const double* in, int64_t ldi, double* out, int64_t ldo, int64_t n, int64_t nrhs, hipStream_t st) {
  if (n * nrhs > 0)
    hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, ldi, out, ldo, n, nrhs);
}

}  // namespace h2
