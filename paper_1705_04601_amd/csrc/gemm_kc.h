// Batched, segmented small GEMM on MFMA (gemm_kc_kernel) and the launch of
// its instances by output tile shape; included by one translation unit per
// role so that the instances compile side by side.
#pragma once

#include "device_common.h"

namespace h2 {
namespace {

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

// Operand fetch of the direct kernel for one 16-row (or 16-column) block and
// the four k of this lane: K-contiguous rows (vector load) or M-contiguous
// columns (one load per k, coalesced across the 16 lanes of a group).
// Generated operands go through gen4.
template <class T, int MODE>
__device__ __forceinline__ void fetch4(const T* p, int64_t ld, int row, int k, int K, bool ok, T* v) {
  if (MODE == 0) {          // element (row, k) at p[k + row ld]
    load4<T>(p, k, K, ok, v);
  } else {                  // element (row, k) at p[row + k ld]
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = (ok && k + s < K) ? p[row + int64_t(k + s) * ld] : T(0);
  }
}

// Generated operand block for the four k of this lane: the kernel of KERN
// (kernel_value) at x_row - y_k, dg on the diagonal, from
// the row's point, held in registers for the whole
// segment, and the chunk's four source points, loaded once per chunk and
// shared by every block of the tile.  Coordinates past dim are zero on both
// sides; the sum runs over a = 0 .. dim - 1 in order (kernel_blocks_kernel
// forms the same values).
template <class T, int KERN>
__device__ __forceinline__ void gen4(const double (&prow)[3], const double (&pcol)[4][3], int row, int k, int K,
                                     bool ok, int dim, double scale, double dg, double param, bool diag, T* v) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    T val = T(0);
    if (ok && k + s < K) {
      if (diag && row == k + s) {
        val = T(dg);
      } else {
        double d2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
          if (a < dim) {
            const double d = prow[a] - pcol[s][a];
            d2 += d * d;
          }
        val = T(kernel_value<KERN>(d2, scale, param));
      }
    }
    v[s] = val;
  }
}

// acc += op(A) op(B) for one segment; AM / BM select the fetch of each operand.
template <class T, int AM, int BM, int MB, int NB, int KERN>
__device__ __forceinline__ void direct_segment(typename Mfma<T>::V (&acc)[MB][NB], int nbm, int nbn,
                                               const GemmSeg& sg, int m0, int n0, int M, int N, int lane,
                                               int dim, double scale, double dg, double param) {
  const int r = lane % 16, kq = 4 * (lane / 16);
  const T* A = static_cast<const T*>(sg.A);
  const T* B = static_cast<const T*>(sg.B);
  const double* pr = static_cast<const double*>(sg.A);
  const int K = sg.K;
  const T* pa[MB];
  const T* pb[NB];
  int ra[MB], cb[NB];
  bool oa[MB], ob[NB];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    ra[b] = m0 + 16 * b + r;
    oa[b] = b < nbm && ra[b] < M;
    pa[b] = (AM == 0) ? A + int64_t(oa[b] ? ra[b] : 0) * sg.lda : A;
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    cb[b] = n0 + 16 * b + r;
    ob[b] = b < nbn && cb[b] < N;
    pb[b] = (BM == 0) ? B + int64_t(ob[b] ? cb[b] : 0) * sg.ldb : B;  // BM 1, 2: addressed per element
  }
  // generated operands: the points of this lane's rows (A) or columns (B)
  constexpr int GA = AM == 2 ? MB : 1, GB = BM == 2 ? NB : 1;
  double prA[GA][3], prB[GB][3];
  if (AM == 2) {
#pragma unroll
    for (int b = 0; b < GA; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) prA[b][a] = (oa[b] && a < dim) ? pr[ra[b] * dim + a] : 0.0;
  }
  if (BM == 2) {
    const double* pcb = static_cast<const double*>(sg.B);
#pragma unroll
    for (int b = 0; b < GB; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) prB[b][a] = (ob[b] && a < dim) ? pcb[cb[b] * dim + a] : 0.0;
  }
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int k = k0 + kq;
    T a[MB][4], bv[NB][4];
    double pcol[4][3];
    if (AM == 2 || BM == 2) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) pcol[s][a] = (k + s < K && a < dim) ? sg.pc[(k + s) * dim + a] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < MB; ++b)
      if (b < nbm) {
        if constexpr (AM == 2) gen4<T, KERN>(prA[b], pcol, ra[b], k, K, oa[b], dim, scale, dg, param, sg.diag, a[b]);
        else fetch4<T, AM>(pa[b], sg.lda, ra[b], k, K, oa[b], a[b]);
      }
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b < nbn) {
        if constexpr (BM == 2) gen4<T, KERN>(prB[b], pcol, cb[b], k, K, ob[b], dim, scale, dg, param, sg.diag, bv[b]);
        else fetch4<T, BM>(pb[b], sg.ldb, cb[b], k, K, ob[b], bv[b]);
      }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int bm = 0; bm < MB; ++bm)
#pragma unroll
        for (int bn = 0; bn < NB; ++bn)
          if (bm < nbm && bn < nbn) acc[bm][bn] = Mfma<T>::run(bv[bn][s], a[bm][s], acc[bm][bn]);
  }
}

// Pipelined path of the stored layouts with A M-contiguous (the solve sweeps:
// A is a block of right-hand sides, element (m, k) at A[m + k lda]; B is a
// block of S or Q_t, K-contiguous (BM 0: (k, n) at B[k + n ldb]) or
// N-contiguous (BM 1: (k, n) at B[n + k ldb])).  The item's (segment, 16-wide
// k step) pairs form one chunk stream read through two register sets: the
// loads of the next chunk are in flight while the MFMAs of the current one
// issue.  Every chunk issues the same loads, through buffer resources that
// start at the chunk: reads past the segment's K rows of A, past the block's
// end or of a chunk beyond the item's last segment (a resource of size zero)
// return zero and move no memory; a B read past K inside the block meets zero
// rows of A.  Blocks of the tile outside the item read at an offset outside
// every resource.  The sums run in the same order as direct_segment's, so
// both give the same bits.  Segment descriptors are loaded 64 at a time, one
// per lane, and taken out with readlane, so that moving to the next segment
// waits for no memory.
template <class T, int BM, int MB, int NB>
struct PipeCursor {
  static constexpr int BL = BM == 0 ? 1 : 4;  // B loads per block and chunk
  int si, se, k0;
  bool valid;
  int dbase;                       // lane l holds the descriptor of segment dbase + l
  uint32_t d[7];                   // A (2 words), B (2), K, lda, ldb
  const T* A;                      // the current segment (wave-uniform)
  const T* B;
  int K, lda, ldb;
  uint32_t oa[MB][4], ob[NB][BL];  // lane offsets inside a chunk (bytes), fixed per segment
};

// Descriptors of segments dbase .. dbase + 63, one per lane (vector loads, so
// that a segment switch reads registers only).
template <class T, int BM, int MB, int NB>
__device__ __forceinline__ void pipe_load_desc(PipeCursor<T, BM, MB, NB>& c, const GemmSeg* segs, int lane) {
  static_assert(sizeof(GemmSeg) == 40, "descriptor layout: A, B, pc, K, lda, ldb, flags");
  const int i = c.dbase + lane < c.se ? c.dbase + lane : c.se - 1;
  const uint32_t* w = reinterpret_cast<const uint32_t*>(segs + i);
  const uint2 ab0 = *reinterpret_cast<const uint2*>(w);
  const uint2 ab1 = *reinterpret_cast<const uint2*>(w + 2);
  const uint2 kl = *reinterpret_cast<const uint2*>(w + 6);
  c.d[0] = ab0.x;
  c.d[1] = ab0.y;
  c.d[2] = ab1.x;
  c.d[3] = ab1.y;
  c.d[4] = kl.x;
  c.d[5] = kl.y;
  c.d[6] = w[8];
}

// The current segment's fields and lane offsets (blocks outside the item:
// kOutside).
template <class T, int BM, int MB, int NB>
__device__ __forceinline__ void pipe_setup(PipeCursor<T, BM, MB, NB>& c, int m0, int n0, int nbm, int nbn, int r,
                                           int kq) {
  const int idx = c.si - c.dbase;
  auto rd = [&](int k) { return uint32_t(__builtin_amdgcn_readlane(int(c.d[k]), idx)); };
  c.A = reinterpret_cast<const T*>((uint64_t(rd(1)) << 32) | rd(0));
  c.B = reinterpret_cast<const T*>((uint64_t(rd(3)) << 32) | rd(2));
  c.K = int(rd(4));
  c.lda = int(rd(5));
  c.ldb = int(rd(6));
  const int lda = c.lda, ldb = c.ldb;
#pragma unroll
  for (int q = 0; q < MB; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s)
      c.oa[q][s] = q < nbm ? uint32_t((kq + s) * lda + m0 + 16 * q + r) * uint32_t(sizeof(T)) : kOutside;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if constexpr (BM == 0) {
      c.ob[q][0] = q < nbn ? uint32_t((n0 + 16 * q + r) * ldb + kq) * uint32_t(sizeof(T)) : kOutside;
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        c.ob[q][s] = q < nbn ? uint32_t((kq + s) * ldb + n0 + 16 * q + r) * uint32_t(sizeof(T)) : kOutside;
    }
  }
}

template <class T, int BM, int MB, int NB>
__device__ __forceinline__ void pipe_next(PipeCursor<T, BM, MB, NB>& c, const GemmSeg* segs, int m0, int n0,
                                          int nbm, int nbn, int r, int kq, int lane) {
  if (!c.valid) return;
  c.k0 += 16;
  if (c.k0 < c.K) return;
  c.k0 = 0;
  if (++c.si >= c.se) {
    c.valid = false;
    return;
  }
  // the descriptor reload waits for every load in flight: a path of its own,
  // so that the common one does not inherit the wait
  if (c.si - c.dbase >= 64) {
    c.dbase += 64;
    pipe_load_desc(c, segs, lane);
    pipe_setup(c, m0, n0, nbm, nbn, r, kq);
  } else {
    pipe_setup(c, m0, n0, nbm, nbn, r, kq);
  }
}

// The same loads for every chunk: resources start at the chunk (A: k0 rows
// on, B: k0 on along K) and end with the segment's block.
template <class T, int BM, int MB, int NB>
__device__ __forceinline__ void pipe_fetch(const PipeCursor<T, BM, MB, NB>& c, int N, T (&a)[MB][4],
                                           T (&b)[NB][4]) {
  const int K = c.K, lda = c.lda, ldb = c.ldb, k0 = c.k0;
  const uint32_t na = c.valid ? uint32_t((K - k0) * lda) * uint32_t(sizeof(T)) : 0u;
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(c.A + int64_t(k0) * lda, na);
#pragma unroll
  for (int q = 0; q < MB; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s) a[q][s] = BufLoad1<T>::run(ra, c.oa[q][s]);
  if constexpr (BM == 0) {
    const uint32_t nb = c.valid ? uint32_t(N * ldb - k0) * uint32_t(sizeof(T)) : 0u;
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(c.B + k0, nb);
#pragma unroll
    for (int q = 0; q < NB; ++q) BufLoad4<T>::run(rb, c.ob[q][0], b[q]);
  } else {
    const uint32_t nb = c.valid ? uint32_t((K - k0) * ldb) * uint32_t(sizeof(T)) : 0u;
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(c.B + int64_t(k0) * ldb, nb);
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) b[q][s] = BufLoad1<T>::run(rb, c.ob[q][s]);
  }
}

// Column blocks outside the item (zero operands, never stored) are skipped
// with one wave-uniform branch each; rows are not (the right-hand sides fill
// the row tiles).
template <class T, int MB, int NB>
__device__ __forceinline__ void pipe_mfma(typename Mfma<T>::V (&acc)[MB][NB], const T (&a)[MB][4],
                                          const T (&b)[NB][4], int nbn) {
#pragma unroll
  for (int bn = 0; bn < NB; ++bn)
    if (bn == 0 || bn < nbn) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int bm = 0; bm < MB; ++bm) acc[bm][bn] = Mfma<T>::run(b[bn][s], a[bm][s], acc[bm][bn]);
    }
}

// Two register sets: the loop multiplies one chunk while the next one's
// loads are in flight, and leaves once per two chunks; a chunk past the
// item's end reads zeros, so multiplying it adds nothing.
template <class T, int BM, int MB, int NB>
__device__ __forceinline__ void pipe_item(typename Mfma<T>::V (&acc)[MB][NB], const GemmLaunch& g,
                                          const GemmItem& it, int m0, int n0, int nbm, int nbn, int lane) {
  if (it.seg_begin >= it.seg_end) return;
  const int r = lane % 16, kq = 4 * (lane / 16);
  PipeCursor<T, BM, MB, NB> c;
  c.si = it.seg_begin;
  c.se = it.seg_end;
  c.k0 = 0;
  c.valid = true;
  c.dbase = c.si;
  pipe_load_desc(c, g.segs, lane);
  pipe_setup(c, m0, n0, nbm, nbn, r, kq);
  T a[2][MB][4], b[2][NB][4];
  pipe_fetch(c, it.N, a[0], b[0]);
  while (true) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      pipe_next(c, g.segs, m0, n0, nbm, nbn, r, kq, lane);
      pipe_fetch(c, it.N, a[1 - i], b[1 - i]);
      __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
      pipe_mfma<T, MB, NB>(acc, a[i], b[i], nbn);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (!c.valid) break;
  }
  // set 0 holds a chunk fetched but not yet multiplied (zeros when past the end)
  pipe_mfma<T, MB, NB>(acc, a[0], b[0], nbn);
}

// AM / BM: operand layouts of every segment of the launch (see direct_segment);
// the tile is MB x NB blocks of 16 x 16; KERN: kernel of generated operands
// (GemmItem::gkern, one for the whole launch)
// The solve sweeps run g.wg_rows waves per work-group, wave w on row tile
// (tile row) wg_rows + w of the same tile column; other roles one wave.
template <class T, int ROLE, int AM, int BM, int MB, int NB, int KERN>
__global__ __launch_bounds__(ROLE == ROLE_SOLVE ? 64 * kSolveWaves : 64)
__attribute__((amdgpu_waves_per_eu(MB * NB * int(sizeof(T)) >= 128 ? 2 : 1))) void gemm_kc_kernel(GemmLaunch g) {
  using V = typename Mfma<T>::V;
  const int lane = threadIdx.x % 64;
  // the solve and matvec lists interleave heavy and light items: keep their
  // round-robin spread over the XCDs
  const int tb = (ROLE == ROLE_TRANSFORM || ROLE == ROLE_FACTOR) ? xcd_tile(blockIdx.x, gridDim.x) : int(blockIdx.x);
  const uint32_t code = static_cast<uint32_t>(g.tiles[tb]);
  const GemmItem it = g.items[code >> 8];
  const int trow = ROLE == ROLE_SOLVE ? int((code >> 4) & 15) * g.wg_rows + int(threadIdx.x / 64)
                                      : int((code >> 4) & 15);
  const int m0 = trow * 16 * MB, n0 = int(code & 15) * 16 * NB;
  if (m0 >= it.M) return;  // a wave past the last row tile (no barriers follow)
  const int nbm = min(MB, (it.M - m0 + 15) / 16), nbn = min(NB, (it.N - n0 + 15) / 16);
  V acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = V{0, 0, 0, 0};
  if constexpr (ROLE == ROLE_SOLVE && AM == 1 && BM != 2) {
    pipe_item<T, BM, MB, NB>(acc, g, it, m0, n0, nbm, nbn, lane);
  } else {
    for (int si = it.seg_begin; si < it.seg_end; ++si) {
      const GemmSeg sg = g.segs[si];
      direct_segment<T, AM, BM, MB, NB, KERN>(acc, nbm, nbn, sg, m0, n0, it.M, it.N, lane, it.gdim, it.gscale, it.gdiag,
                                              it.gparam);
    }
  }
#pragma unroll
  for (int bm = 0; bm < MB; ++bm)
#pragma unroll
    for (int bn = 0; bn < NB; ++bn) {
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


// Launch of one built instance: variant V of a role and layout pair (a
// variant that is not built launches nothing; the host plans only built ones).
template <class T, int ROLE, int AM, int BM, int V>
void launch_variant(const GemmLaunch& g, hipStream_t st) {
  constexpr int code = gemm_shape(sizeof(T) == 4 ? 1 : 0, ROLE, AM, BM, V);
  if constexpr (code != 0) {
    constexpr int MB = code >> 4, NB = code & 15;
    if constexpr (AM == 2 || BM == 2) {
      if (g.kern == 1) {
        hipLaunchKernelGGL((gemm_kc_kernel<T, ROLE, AM, BM, MB, NB, 1>), dim3(g.ntiles), dim3(ROLE == ROLE_SOLVE ? 64 * g.wg_rows : 64), 0, st, g);
        return;
      }
      if (g.kern == 2) {
        hipLaunchKernelGGL((gemm_kc_kernel<T, ROLE, AM, BM, MB, NB, 2>), dim3(g.ntiles), dim3(ROLE == ROLE_SOLVE ? 64 * g.wg_rows : 64), 0, st, g);
        return;
      }
    }
    hipLaunchKernelGGL((gemm_kc_kernel<T, ROLE, AM, BM, MB, NB, 0>), dim3(g.ntiles), dim3(ROLE == ROLE_SOLVE ? 64 * g.wg_rows : 64), 0, st, g);
  }
}

template <class T, int ROLE, int AM, int BM>
void launch_layout(const GemmLaunch& g, hipStream_t st) {
  switch (g.variant) {
    case 1: return launch_variant<T, ROLE, AM, BM, 1>(g, st);
    case 2: return launch_variant<T, ROLE, AM, BM, 2>(g, st);
    case 3: return launch_variant<T, ROLE, AM, BM, 3>(g, st);
    case 4: return launch_variant<T, ROLE, AM, BM, 4>(g, st);
    case 5: return launch_variant<T, ROLE, AM, BM, 5>(g, st);
    default: return launch_variant<T, ROLE, AM, BM, 0>(g, st);
  }
}

}  // namespace
}  // namespace h2
