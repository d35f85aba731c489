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

// Pipelined path of the stored layouts with A M-contiguous (the solve sweeps,
// where A is a block of right-hand sides and B a block of S or Q_t, and the
// transforms of that layout): element (m, k) of A at A[m + k lda]; B
// K-contiguous (BM 0: (k, n) at B[k + n ldb]) or N-contiguous (BM 1: (k, n) at
// B[n + k ldb]).  The item's (segment, 16-wide
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
template <class T, int BM, int MB, int NB, int AM = 1>
struct PipeCursor {
  static constexpr int AL = AM == 0 ? 1 : 4;  // A loads per block and chunk
  static constexpr int BL = BM == 0 ? 1 : 4;  // B loads per block and chunk
  int si, se, k0;
  bool valid;
  int dbase;                       // lane l holds the descriptor of segment dbase + l
  uint32_t d[7];                   // A (2 words), B (2), K, lda, ldb
  const T* A;                      // the current segment (wave-uniform)
  const T* B;
  int K, lda, ldb;
  uint32_t oa[MB][AL], ob[NB][BL];  // lane offsets inside a chunk (bytes), fixed per segment
};

// Descriptors of segments dbase .. dbase + 63, one per lane (vector loads, so
// that a segment switch reads registers only).
template <class T, int BM, int MB, int NB, int AM>
__device__ __forceinline__ void pipe_load_desc(PipeCursor<T, BM, MB, NB, AM>& c, const GemmSeg* segs, int lane) {
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
template <class T, int BM, int MB, int NB, int AM>
__device__ __forceinline__ void pipe_setup(PipeCursor<T, BM, MB, NB, AM>& c, int m0, int n0, int nbm, int nbn, int r,
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
  for (int q = 0; q < MB; ++q) {
    if constexpr (AM == 0) {
      c.oa[q][0] = q < nbm ? uint32_t((m0 + 16 * q + r) * lda + kq) * uint32_t(sizeof(T)) : kOutside;
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        c.oa[q][s] = q < nbm ? uint32_t((kq + s) * lda + m0 + 16 * q + r) * uint32_t(sizeof(T)) : kOutside;
    }
  }
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

template <class T, int BM, int MB, int NB, int AM>
__device__ __forceinline__ void pipe_next(PipeCursor<T, BM, MB, NB, AM>& c, const GemmSeg* segs, int m0, int n0,
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
template <class T, int BM, int MB, int NB, int AM>
__device__ __forceinline__ void pipe_fetch(const PipeCursor<T, BM, MB, NB, AM>& c, int M, int N, int kq,
                                           T (&a)[MB][4], T (&b)[NB][4]) {
  const int K = c.K, lda = c.lda, ldb = c.ldb, k0 = c.k0;
  if constexpr (AM == 0) {
    // A K-contiguous ((m, k) at A[k + m lda]): four k of a row per load, k
    // past K inside a row read as zero
    const uint32_t na = c.valid ? uint32_t(M * lda - k0) * uint32_t(sizeof(T)) : 0u;
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(c.A + k0, na);
    const int kr = K - k0 - kq;
#pragma unroll
    for (int q = 0; q < MB; ++q) {
      BufLoad4<T>::run(ra, c.oa[q][0], a[q]);
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) a[q][s2] = s2 < kr ? a[q][s2] : T(0);
    }
  } else {
    const uint32_t na = c.valid ? uint32_t((K - k0) * lda) * uint32_t(sizeof(T)) : 0u;
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(c.A + int64_t(k0) * lda, na);
#pragma unroll
    for (int q = 0; q < MB; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) a[q][s] = BufLoad1<T>::run(ra, c.oa[q][s]);
  }
  if constexpr (BM == 0) {
    const uint32_t nb = c.valid ? uint32_t(N * ldb - k0) * uint32_t(sizeof(T)) : 0u;
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(c.B + k0, nb);
    // k past K inside a column (when ldb > K) is storage outside the block,
    // whatever it holds: read as zero
    const int kr = K - k0 - kq;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      BufLoad4<T>::run(rb, c.ob[q][0], b[q]);
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) b[q][s2] = s2 < kr ? b[q][s2] : T(0);
    }
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
template <class T, int AM, int BM, int MB, int NB>
__device__ __forceinline__ void pipe_item(typename Mfma<T>::V (&acc)[MB][NB], const GemmLaunch& g,
                                          const GemmItem& it, int m0, int n0, int nbm, int nbn, int lane) {
  if (it.seg_begin >= it.seg_end) return;
  const int r = lane % 16, kq = 4 * (lane / 16);
  PipeCursor<T, BM, MB, NB, AM> c;
  c.si = it.seg_begin;
  c.se = it.seg_end;
  c.k0 = 0;
  c.valid = true;
  c.dbase = c.si;
  pipe_load_desc(c, g.segs, lane);
  pipe_setup(c, m0, n0, nbm, nbn, r, kq);
  T a[2][MB][4], b[2][NB][4];
  pipe_fetch(c, it.M, it.N, kq, a[0], b[0]);
  while (true) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      pipe_next(c, g.segs, m0, n0, nbm, nbn, r, kq, lane);
      pipe_fetch(c, it.M, it.N, kq, a[1 - i], b[1 - i]);
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
  if constexpr (((ROLE == ROLE_SOLVE || ROLE == ROLE_TRANSFORM) && AM == 1 && BM != 2) ||
                ((ROLE == ROLE_TRANSFORM || ROLE == ROLE_FACTOR) && AM == 0 && BM == 0)) {
    pipe_item<T, AM, BM, MB, NB>(acc, g, it, m0, n0, nbm, nbn, lane);
  } else {
    for (int si = it.seg_begin; si < it.seg_end; ++si) {
      const GemmSeg sg = g.segs[si];
      direct_segment<T, AM, BM, MB, NB, KERN>(acc, nbm, nbn, sg, m0, n0, it.M, it.N, lane, it.gdim, it.gscale, it.gdiag,
                                              it.gparam);
    }
  }
  const int mode = it.store ? int(GEMM_STORE) : g.mode;
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
        store_out<T>(it, q, lr, lc, val, mode);
        if (q == 0) store_out<T>(it, 4, lr, lc, val, mode);
      }
    }
}



// LDS-staged solve tile (FP32): the work-group's W waves cover W x 32 rows (the
// right-hand sides) of one column tile of NB blocks of 16.  Each 16-wide k
// step of the item's chunk stream is loaded once for the whole work-group,
// A (the right-hand-side block, m-contiguous) into sA[k][m] and B (the S or
// Q_t block) into sB[n][k], with the same buffer resources as pipe_fetch
// (reads past a block return zero); the next step's loads are in flight
// while the waves multiply the current one out of LDS, and one barrier per
// step hands the buffers over.  Lane (r, g) reads the same k = 4 g + s of the
// same rows and columns as the other solve kernels, so the sums run in the
// same order.  Waves whose rows lie past the item load and wait like the
// others but compute nothing.
constexpr int kLdsAS = 132;  // sA row stride (words): 4 k rows apart land 16 banks apart
constexpr int kLdsBS = 20;   // sB row stride (words): 16 k + 4, rows 16-byte aligned

template <int BM, int NB, int W>
struct LdsStage {
  static constexpr int NA = 2;                        // float4 loads of A per thread
  static constexpr int NBL = (64 * NB + 64 * W - 1) / (64 * W);  // float4 loads of B per thread
  f4 a[NA];
  f4 b[NBL];
};

template <int BM, int NB, int W>
__device__ __forceinline__ void lds_fetch(const PipeCursor<float, BM, 2, NB>& c, int mg0, int n0, int N, int tid,
                                          LdsStage<BM, NB, W>& r) {
  constexpr int T = 64 * W;
  const int K = c.K, lda = c.lda, ldb = c.ldb, k0 = c.k0;
  const uint32_t na = c.valid ? uint32_t((K - k0) * lda) * 4u : 0u;
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(c.A + int64_t(k0) * lda, na);
#pragma unroll
  for (int j = 0; j < LdsStage<BM, NB, W>::NA; ++j) {
    const int f = tid + j * T;  // 16 k rows of 8 W float4
    const int k = f / (8 * W), mq = f % (8 * W);
    r.a[j] = raw_buffer_load_f4(ra, int(uint32_t(k * lda + mg0 + 4 * mq) * 4u), 0, 0);
  }
  if constexpr (BM == 0) {
    const uint32_t nb = c.valid ? uint32_t(N * ldb - k0) * 4u : 0u;
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(c.B + k0, nb);
#pragma unroll
    for (int j = 0; j < LdsStage<BM, NB, W>::NBL; ++j) {
      const int f = tid + j * T;  // NB 16 columns of 4 float4
      const int col = f / 4, kq4 = f % 4;
      const uint32_t off = f < 64 * NB ? uint32_t((n0 + col) * ldb + 4 * kq4) * 4u : kOutside;
      r.b[j] = raw_buffer_load_f4(rb, int(off), 0, 0);
    }
  } else {
    const uint32_t nb = c.valid ? uint32_t((K - k0) * ldb) * 4u : 0u;
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(c.B + int64_t(k0) * ldb, nb);
#pragma unroll
    for (int j = 0; j < LdsStage<BM, NB, W>::NBL; ++j) {
      const int f = tid + j * T;  // 16 k rows of 4 NB float4
      const int k = f / (4 * NB), nq = f % (4 * NB);
      const uint32_t off = f < 64 * NB ? uint32_t(k * ldb + n0 + 4 * nq) * 4u : kOutside;
      r.b[j] = raw_buffer_load_f4(rb, int(off), 0, 0);
    }
  }
}

template <int BM, int NB, int W>
__device__ __forceinline__ void lds_store(const LdsStage<BM, NB, W>& r, float* sA, float* sB, int tid) {
  constexpr int T = 64 * W;
#pragma unroll
  for (int j = 0; j < LdsStage<BM, NB, W>::NA; ++j) {
    const int f = tid + j * T;
    const int k = f / (8 * W), mq = f % (8 * W);
    *reinterpret_cast<f4*>(sA + k * kLdsAS + 4 * mq) = r.a[j];
  }
#pragma unroll
  for (int j = 0; j < LdsStage<BM, NB, W>::NBL; ++j) {
    const int f = tid + j * T;
    if (f < 64 * NB) {
      if constexpr (BM == 0) {
        const int col = f / 4, kq4 = f % 4;
        *reinterpret_cast<f4*>(sB + col * kLdsBS + 4 * kq4) = r.b[j];
      } else {
        const int k = f / (4 * NB), nq = f % (4 * NB);
#pragma unroll
        for (int e = 0; e < 4; ++e) sB[(4 * nq + e) * kLdsBS + k] = r.b[j][e];
      }
    }
  }
}

template <int NB>
__device__ __forceinline__ void lds_mfma(f4 (&acc)[2][NB], const float* sA, const float* sB, int wrow, int lane,
                                         int nbn) {
  const int r = lane % 16, g = lane / 16;
  float a[2][4];
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int s = 0; s < 4; ++s) a[bm][s] = sA[(4 * g + s) * kLdsAS + wrow + 16 * bm + r];
#pragma unroll
  for (int bn = 0; bn < NB; ++bn)
    if (bn == 0 || bn < nbn) {
      const f4 b = *reinterpret_cast<const f4*>(sB + (16 * bn + r) * kLdsBS + 4 * g);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int bm = 0; bm < 2; ++bm) acc[bm][bn] = Mfma<float>::run(b[s], a[bm][s], acc[bm][bn]);
    }
}

template <int BM, int NB, int W>
__global__ __launch_bounds__(64 * W) void gemm_solve_lds_kernel(GemmLaunch g) {
  __shared__ __attribute__((aligned(16))) float sA[2][16 * kLdsAS];
  __shared__ __attribute__((aligned(16))) float sB[2][16 * NB * kLdsBS];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const uint32_t code = static_cast<uint32_t>(g.tiles[blockIdx.x]);
  const GemmItem it = g.items[code >> 8];
  const int mg0 = int((code >> 4) & 15) * W * 32;
  const int m0 = mg0 + 32 * wave, n0 = int(code & 15) * 16 * NB;
  const int nbm = m0 < it.M ? min(2, (it.M - m0 + 15) / 16) : 0;
  const int nbn = min(NB, (it.N - n0 + 15) / 16);
  f4 acc[2][NB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f4{0, 0, 0, 0};
  if (it.seg_begin < it.seg_end) {
    const int r = lane % 16, kq = 4 * (lane / 16);
    PipeCursor<float, BM, 2, NB> c;
    c.si = it.seg_begin;
    c.se = it.seg_end;
    c.k0 = 0;
    c.valid = true;
    c.dbase = c.si;
    pipe_load_desc(c, g.segs, lane);
    pipe_setup(c, m0, n0, 2, nbn, r, kq);  // the scalars; the lane offsets go unused here
    LdsStage<BM, NB, W> st;
    lds_fetch<BM, NB, W>(c, mg0, n0, it.N, tid, st);
    lds_store<BM, NB, W>(st, sA[0], sB[0], tid);
    __syncthreads();
    for (int buf = 0;; buf ^= 1) {
      pipe_next(c, g.segs, m0, n0, 2, nbn, r, kq, lane);
      const bool more = c.valid;
      lds_fetch<BM, NB, W>(c, mg0, n0, it.N, tid, st);
      if (nbm > 0) lds_mfma<NB>(acc, sA[buf], sB[buf], 32 * wave, lane, nbn);
      if (!more) break;
      lds_store<BM, NB, W>(st, sA[buf ^ 1], sB[buf ^ 1], tid);
      __syncthreads();
    }
  }
  const int mode = it.store ? int(GEMM_STORE) : g.mode;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < NB; ++bn) {
      if (bm >= nbm || bn >= nbn) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + 16 * bm + lane % 16;
        const int col = n0 + 16 * bn + Mfma<float>::row(lane, v);
        if (row >= it.M || col >= it.N) continue;
        const int q = (row >= it.rs ? 2 : 0) + (col >= it.cs ? 1 : 0);
        const int lr = row - (q >= 2 ? it.rs : 0), lc = col - ((q & 1) ? it.cs : 0);
        const float val = acc[bm][bn][v];
        store_out<float>(it, q, lr, lc, val, mode);
        if (q == 0) store_out<float>(it, 4, lr, lc, val, mode);
      }
    }
}

// Launch of one built instance: variant V of a role and layout pair (a
// variant that is not built launches nothing; the host plans only built ones).
template <class T, int ROLE, int AM, int BM, int V>
void launch_variant(const GemmLaunch& g, hipStream_t st) {
  constexpr int code = gemm_shape(sizeof(T) == 4 ? 1 : 0, ROLE, AM, BM, V);
  if constexpr (code != 0 && (code & kGemmLds) != 0) {
    if constexpr (ROLE == ROLE_SOLVE && AM == 1 && BM != 2 && sizeof(T) == 4 && ((code >> 4) & 15) == 2) {
      constexpr int NB = code & 15;
      switch (g.wg_rows) {
        case 1: hipLaunchKernelGGL((gemm_solve_lds_kernel<BM, NB, 1>), dim3(g.ntiles), dim3(64), 0, st, g); break;
        case 2: hipLaunchKernelGGL((gemm_solve_lds_kernel<BM, NB, 2>), dim3(g.ntiles), dim3(128), 0, st, g); break;
        case 3: hipLaunchKernelGGL((gemm_solve_lds_kernel<BM, NB, 3>), dim3(g.ntiles), dim3(192), 0, st, g); break;
        default: hipLaunchKernelGGL((gemm_solve_lds_kernel<BM, NB, 4>), dim3(g.ntiles), dim3(256), 0, st, g); break;
      }
    }
  } else if constexpr (code != 0) {
    constexpr int MB = (code >> 4) & 15, NB = code & 15;
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
