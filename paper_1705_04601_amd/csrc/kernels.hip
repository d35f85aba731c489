// HIP kernels of libh2sp for gfx950 (CDNA4, 64-wide wavefronts).
//
//  * gemm_kc_kernel: batched, segmented small GEMM on MFMA (v_mfma_f64_16x16x4
//    / v_mfma_f32_16x16x4).  One wavefront per output tile (32 x 32, 64 x 32
//    or 64 x 64 by role and operand layout), operands
//    straight from L2 without LDS; either operand can be generated on the fly
//    from points (kernel evaluation, so a generated block never touches HBM); the
//    epilogue scatters the four quadrants of the tile to separate
//    destinations (the basis / non-basis split of Section 2).
//  * schur_kernel: the Schur updates of the block factorisation.
//  * qr_kernel: Householder QR of a cluster basis held in LDS, FP64, norms by
//    wavefront reductions, explicit square Q (Section 4.2).
//  * inverse_kernel: FP64 Gauss-Jordan inversion with partial pivoting of a
//    pivot block of S, LDS resident.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_common.h"
#include "kernels.h"

namespace h2 {

// The scratch array of the allocation-free entry point.  Host code reaches it
// only through its device address (noalloc_scratch), never by its name, which
// on the host is a stand-in and not a device address.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

namespace {

// Schur update of the block factorisation with compact descriptors:
// S[out] (M x N, ld M) -= sum_seg Z[a]^T (K x M, ld K16) S[b] (K x N, ld K),
// K16 = K rounded up to 16.  One wave per 64 x 64 tile.  The (segment,
// 16-wide k step) pairs form one chunk stream, consumed through a ring of NS
// register sets: the loads of NS - 1 chunks are in flight while the MFMAs of
// the oldest issue.  The number of 16 x 16 blocks of the tile (NBM x NBN) is a
// template parameter and every load is issued unconditionally, so the count
// of loads in flight is static and the compiler waits only for the oldest set.
//
// Operands are read with buffer loads: per segment, one resource (base and
// size in bytes) for the Z_ki block and one for the S_kj block, and one 32-bit
// offset per lane and 16 x 16 block that stays fixed for the whole segment; a
// chunk only moves the two bases on by one row of tiles (16 k).  Reads outside
// a resource return zero, which covers a chunk past the item's last segment (a
// resource of size zero); rows past M and columns past N are the zero padding
// of the tiles.  A lane whose four k start
// at or past K reads through an offset outside both resources (zero, and no
// memory traffic); in the lane that holds K itself, k past K meets the zero
// rows of the padded Z_ki, and the S_kj operand reads the next column of the
// block, or zero past the block's end.
// Segment descriptors are loaded 64 at a time, one per lane, and taken out
// with readlane, so that moving to the next segment waits for no memory.
// Chunk cursor of a tile (wave-uniform apart from the lane offsets and the
// lane-held descriptors).
template <class T, int NBM, int NBN>
struct SchurCursor {
  int si, se, k0, K;
  bool valid;           // false past the item's last segment (and stays false)
  int dbase;            // lane l holds the descriptor of segment dbase + l
  uint32_t d[4];
  const T* pa;          // Z_ki and S_kj of the current segment
  const T* pb;
  uint32_t na, nb;      // their sizes in bytes
  int sha;              // elements the Z_ki base moves per k (16 per 16-column block)
  int shb;              // elements the S_kj base moves per k (as for Z_ki in tiles, 1 in place)
  uint32_t oa[NBM], ob[NBN];
};

template <class T, int NBM, int NBN>
__device__ __forceinline__ void schur_load_desc(SchurCursor<T, NBM, NBN>& c, const SchurSeg* segs, int lane) {
  const int i = c.dbase + lane < c.se ? c.dbase + lane : c.se - 1;
  const uint4 x = *reinterpret_cast<const uint4*>(segs + i);
  c.d[0] = x.x;
  c.d[1] = x.y;
  c.d[2] = x.z;
  c.d[3] = x.w;
}

// Operand addressing of one segment.  Z_ki is always in tiles (see
// retile_kernel), lane l's four elements at 4 l inside the tile, so that one
// load instruction reads 1 KB (FP32) of consecutive memory; chunk c of column
// block q lies at (q C + c) 256 elements, C = K16 / 16 (column-outer), or at
// (c Q + q) 256, Q = M16 / 16 (k-outer).  In the k-outer layout blocks of
// consecutive pivots laid out one after the other read as one segment whose
// K is the sum of their padded K (the padding rows are zero).  S_kj is in
// tiles too (the same layout) when the launch says so, else read in place
// (column-major, ld K: each lane reads four consecutive k of its column).
template <class T, int NBM, int NBN>
__device__ __forceinline__ void schur_setup(SchurCursor<T, NBM, NBN>& c, const T* Sb, const T* Z, int tiled_b,
                                            int kouter, int m0, int n0, int M, int N, int r, int kq) {
  static_assert(sizeof(SchurSeg) == 16, "descriptor of four 32-bit words");
  const int idx = c.si - c.dbase;
  const uint64_t b_off = (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(c.d[1]), idx))) << 32) |
                         uint32_t(__builtin_amdgcn_readlane(int(c.d[0]), idx));
  const int a_off = __builtin_amdgcn_readlane(int(c.d[2]), idx);
  const int K = __builtin_amdgcn_readlane(int(c.d[3]), idx);
  const int ck = (K + 15) >> 4;  // chunks of 16 k
  const int lane4 = 4 * (r + 4 * kq);
  c.K = K;
  c.pa = Z + a_off;
  c.pb = Sb + int64_t(b_off);
  c.na = uint32_t(ck * 16 * ((M + 15) & ~15)) * uint32_t(sizeof(T));
  // per 16 k the base moves by one row of tiles (k-outer) or one tile
  c.sha = kouter ? 16 * ((M + 15) >> 4) : 16;
  const int qa = kouter ? 256 : ck * 256;  // elements between column blocks
#pragma unroll
  for (int q = 0; q < NBM; ++q) c.oa[q] = uint32_t((m0 / 16 + q) * qa + lane4) * uint32_t(sizeof(T));
  if (tiled_b) {
    c.shb = kouter ? 16 * ((N + 15) >> 4) : 16;
    c.nb = uint32_t(ck * 16 * ((N + 15) & ~15)) * uint32_t(sizeof(T));
#pragma unroll
    for (int q = 0; q < NBN; ++q) c.ob[q] = uint32_t((n0 / 16 + q) * qa + lane4) * uint32_t(sizeof(T));
  } else {
    c.shb = 1;
    c.nb = uint32_t(K * N) * uint32_t(sizeof(T));
#pragma unroll
    for (int q = 0; q < NBN; ++q) c.ob[q] = uint32_t((n0 + 16 * q + r) * K + kq) * uint32_t(sizeof(T));
  }
}

template <class T, int NBM, int NBN>
__device__ __forceinline__ void schur_next(SchurCursor<T, NBM, NBN>& c, const SchurSeg* segs, const T* Sb,
                                           const T* Z, int tiled_b, int kouter, int m0, int n0, int M, int N, int r,
                                           int kq, int lane) {
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
    schur_load_desc(c, segs, lane);
    schur_setup(c, Sb, Z, tiled_b, kouter, m0, n0, M, N, r, kq);
  } else {
    schur_setup(c, Sb, Z, tiled_b, kouter, m0, n0, M, N, r, kq);
  }
}


// Loads one chunk (the same loads for every chunk, so that the number of
// loads in flight stays static) and returns the MFMA steps it needs: 4 for a
// full chunk, 2 or 1 for the last chunk of a segment with 5..8 or 1..4 valid
// k (see schur_compact), 0 past the item's end.
template <class T, int NBM, int NBN>
__device__ __forceinline__ int schur_fetch(const SchurCursor<T, NBM, NBN>& c, int kq, T (&a)[NBM][4],
                                           T (&b)[NBN][4]) {
  // k0 < K <= K16: both sizes stay positive (a row of tiles moves the base by
  // 16 elements per k and 16-column block, an in-place column block by one)
  const uint32_t sha = uint32_t(c.k0 * c.sha) * uint32_t(sizeof(T));
  const uint32_t shb = uint32_t(c.k0 * c.shb) * uint32_t(sizeof(T));
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(c.pa + c.k0 * c.sha, c.valid ? c.na - sha : 0u);
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(c.pb + c.k0 * c.shb, c.valid ? c.nb - shb : 0u);
  const bool live = c.k0 + kq < c.K;
#pragma unroll
  for (int q = 0; q < NBM; ++q) BufLoad4<T>::run(ra, live ? c.oa[q] : kOutside, a[q]);
#pragma unroll
  for (int q = 0; q < NBN; ++q) BufLoad4<T>::run(rb, live ? c.ob[q] : kOutside, b[q]);
  const int rem = c.K - c.k0;
  return !c.valid ? 0 : rem > 8 ? 4 : rem > 4 ? 2 : 1;
}

// Lane swaps of gfx950 on one operand register (an FP64 value is two).
// swap32: x's lanes 32..63 trade places with y's lanes 0..31 (lane groups 2,
// 3 of x receive groups 0, 1 of y); swap16: x's odd groups trade with y's
// even groups (groups 1, 3 of x receive groups 0, 2 of y).
template <class T>
__device__ __forceinline__ void lane_swap32(T& x, T& y) {
  static_assert(sizeof(T) % 4 == 0, "32-bit words");
  uint32_t u[sizeof(T) / 4], v[sizeof(T) / 4];
  __builtin_memcpy(u, &x, sizeof(T));
  __builtin_memcpy(v, &y, sizeof(T));
#pragma unroll
  for (int w = 0; w < int(sizeof(T) / 4); ++w) {
    const auto r = __builtin_amdgcn_permlane32_swap(u[w], v[w], false, false);
    u[w] = r[0];
    v[w] = r[1];
  }
  __builtin_memcpy(&x, u, sizeof(T));
  __builtin_memcpy(&y, v, sizeof(T));
}
template <class T>
__device__ __forceinline__ void lane_swap16(T& x, T& y) {
  uint32_t u[sizeof(T) / 4], v[sizeof(T) / 4];
  __builtin_memcpy(u, &x, sizeof(T));
  __builtin_memcpy(v, &y, sizeof(T));
#pragma unroll
  for (int w = 0; w < int(sizeof(T) / 4); ++w) {
    const auto r = __builtin_amdgcn_permlane16_swap(u[w], v[w], false, false);
    u[w] = r[0];
    v[w] = r[1];
  }
  __builtin_memcpy(&x, u, sizeof(T));
  __builtin_memcpy(&y, v, sizeof(T));
}

// The last chunk of a segment holds rem < 16 valid k; lane group g holds
// k = 4g + s in register s, so only groups g < ceil(rem / 4) hold data (the
// others read zeros).  With rem <= 8 the data move into fewer registers, the
// same moves for both operands so that every step still pairs equal k:
//   rem 5..8: groups 2, 3 of registers 0, 1 receive registers 2, 3 of groups
//     0, 1; steps 0 and 1 then cover all eight k;
//   rem 1..4: after that, groups 1, 3 of register 0 receive groups 0, 2 of
//     register 1; step 0 covers all four k.
template <class T, int NB>
__device__ __forceinline__ void schur_compact(T (&x)[NB][4], int nsteps) {
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    lane_swap32(x[q][0], x[q][2]);
    lane_swap32(x[q][1], x[q][3]);
    if (nsteps == 1) lane_swap16(x[q][0], x[q][1]);
  }
}

template <class T, int NBM, int NBN>
__device__ __forceinline__ void schur_mfma(typename Mfma<T>::V (&acc)[NBM][NBN], T (&a)[NBM][4], T (&b)[NBN][4],
                                           int nsteps) {
  if (nsteps == 0) return;
  if (nsteps < 4) {
    schur_compact<T, NBM>(a, nsteps);
    schur_compact<T, NBN>(b, nsteps);
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (s >= nsteps) break;
#pragma unroll
    for (int bm = 0; bm < NBM; ++bm)
#pragma unroll
      for (int bn = 0; bn < NBN; ++bn) acc[bm][bn] = Mfma<T>::run(b[bn][s], a[bm][s], acc[bm][bn]);
  }
}

template <class T, int NBM, int NBN, int NS>
__device__ __forceinline__ void schur_tile(const SchurLaunch& g, const SchurItem& it, int m0, int n0, int lane) {
  using V = typename Mfma<T>::V;
  const int r = lane % 16, kq = 4 * (lane / 16);
  T* S = static_cast<T*>(g.S);
  const T* Sb = static_cast<const T*>(g.Sb);
  const T* Z = static_cast<const T*>(g.Z);
  const int tb = g.tiled_b, ko = g.kouter;
  V acc[NBM][NBN];
#pragma unroll
  for (int a = 0; a < NBM; ++a)
#pragma unroll
    for (int b = 0; b < NBN; ++b) acc[a][b] = V{0, 0, 0, 0};
  if (it.seg_begin < it.seg_end) {
    SchurCursor<T, NBM, NBN> c;
    c.si = c.dbase = it.seg_begin;
    c.se = it.seg_end;
    c.k0 = 0;
    c.valid = true;
    schur_load_desc(c, g.segs, lane);
    schur_setup(c, Sb, Z, tb, ko, m0, n0, it.M, it.N, r, kq);
    T a[NS][NBM][4], b[NS][NBN][4];
    int steps[NS];
    steps[0] = schur_fetch(c, kq, a[0], b[0]);
#pragma unroll
    for (int i = 1; i < NS - 1; ++i) {
      schur_next(c, g.segs, Sb, Z, tb, ko, m0, n0, it.M, it.N, r, kq, lane);
      steps[i] = schur_fetch(c, kq, a[i], b[i]);
    }
    // one exit per NS chunks; chunks past the end read zeros and take no step
    while (true) {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        schur_next(c, g.segs, Sb, Z, tb, ko, m0, n0, it.M, it.N, r, kq, lane);
        steps[(i + NS - 1) % NS] = schur_fetch(c, kq, a[(i + NS - 1) % NS], b[(i + NS - 1) % NS]);
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
        schur_mfma<T, NBM, NBN>(acc, a[i], b[i], steps[i]);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (!c.valid) break;
    }
    // sets 0 .. NS - 2 hold chunks fetched but not yet multiplied
#pragma unroll
    for (int i = 0; i < NS - 1; ++i) schur_mfma<T, NBM, NBN>(acc, a[i], b[i], steps[i]);
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

// Tile classes and the depth of the register ring.  Each class runs in a
// kernel of its own, so that each gets the register budget of its own shapes:
//   0: at most 4 blocks of 16 along both sides (FP64: every tile); FP32
//      three sets, FP64 two, two waves per SIMD;
//   1: (FP32) 5 blocks along the longer side, the common whole-target shape
//      of the leaves (65 to 80 rows); two sets, so that the accumulators
//      (at most 100, in AGPRs) and the operands fit two waves per SIMD;
//   2: (FP32) 6 to 8 blocks, up to a whole 128 x 128 target whose 256
//      accumulators fill the AGPRs, one wave per SIMD; as many sets (2 to 4)
//      as fit in about 176 VGPRs, so that the smaller of these shapes keep
//      more chunks in flight.
template <class T, int NBM, int NBN, int CLS>
constexpr int schur_stages() {
  if (CLS == 0) return sizeof(T) == 4 ? 3 : 2;
  if (CLS == 1) return 2;
  constexpr int n = 176 / (4 * (NBM + NBN));
  return n < 2 ? 2 : (n > 4 ? 4 : n);
}

template <class T, int CLS>
__global__ __launch_bounds__(64) void schur_kernel(SchurLaunch g) {
  constexpr int E = schur_edge<T>;
  const int lane = threadIdx.x;
  const uint32_t code = static_cast<uint32_t>(g.tiles[xcd_tile(blockIdx.x, gridDim.x)]);
  const SchurItem it = g.items[code >> 8];
  // a tile row field of 8 or more marks a tile of edge E / 2 (a large target
  // cut into quarters, see schur_tile_code)
  const int fa = int((code >> 4) & 15), fb = int(code & 15);
  const int te = fa >= 8 ? E / 2 : E;
  const int m0 = (fa & 7) * te, n0 = (fb & 7) * te;
  constexpr int B = E / 16;
  const int nbm = min(te / 16, (it.M - m0 + 15) / 16), nbn = min(te / 16, (it.N - n0 + 15) / 16);
#define H2_SCHUR_CASE(I, J) \
  case I * 8 + J: schur_tile<T, I, J, schur_stages<T, I, J, CLS>()>(g, it, m0, n0, lane); break;
  if constexpr (CLS == 0) {
    switch (nbm * 8 + nbn) {
#define H2_SCHUR_ROW(I) H2_SCHUR_CASE(I, 1) H2_SCHUR_CASE(I, 2) H2_SCHUR_CASE(I, 3) H2_SCHUR_CASE(I, 4)
      H2_SCHUR_ROW(1) H2_SCHUR_ROW(2) H2_SCHUR_ROW(3) H2_SCHUR_ROW(4)
#undef H2_SCHUR_ROW
      default: break;
    }
  } else if constexpr (CLS == 1 && B == 8) {
    switch (nbm * 8 + nbn) {
      H2_SCHUR_CASE(5, 1) H2_SCHUR_CASE(5, 2) H2_SCHUR_CASE(5, 3) H2_SCHUR_CASE(5, 4) H2_SCHUR_CASE(5, 5)
      H2_SCHUR_CASE(1, 5) H2_SCHUR_CASE(2, 5) H2_SCHUR_CASE(3, 5) H2_SCHUR_CASE(4, 5)
      default: break;
    }
  } else if constexpr (CLS == 2 && B == 8) {
    switch (nbm * 8 + nbn) {
#define H2_SCHUR_ROW(I) \
  H2_SCHUR_CASE(I, 1) H2_SCHUR_CASE(I, 2) H2_SCHUR_CASE(I, 3) H2_SCHUR_CASE(I, 4) \
  H2_SCHUR_CASE(I, 5) H2_SCHUR_CASE(I, 6) H2_SCHUR_CASE(I, 7) H2_SCHUR_CASE(I, 8)
      H2_SCHUR_ROW(6) H2_SCHUR_ROW(7) H2_SCHUR_ROW(8)
#undef H2_SCHUR_ROW
      H2_SCHUR_CASE(1, 6) H2_SCHUR_CASE(1, 7) H2_SCHUR_CASE(1, 8)
      H2_SCHUR_CASE(2, 6) H2_SCHUR_CASE(2, 7) H2_SCHUR_CASE(2, 8)
      H2_SCHUR_CASE(3, 6) H2_SCHUR_CASE(3, 7) H2_SCHUR_CASE(3, 8)
      H2_SCHUR_CASE(4, 6) H2_SCHUR_CASE(4, 7) H2_SCHUR_CASE(4, 8)
      H2_SCHUR_CASE(5, 6) H2_SCHUR_CASE(5, 7) H2_SCHUR_CASE(5, 8)
      default: break;
    }
  }
#undef H2_SCHUR_CASE
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
__global__ __launch_bounds__(1024) void inverse_kernel(const InvItem<T>* items, int* flag) {
  __shared__ double a[128 * 128];
  __shared__ double fcol[128];
  __shared__ int perm[128];
  const InvItem<T> it = items[blockIdx.x];
  const int m = it.m, tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  // the rank-one update: thread (row r, column group g) owns columns g, g + 16, ...
  const int r = tid % 64, g = tid / 64;
  for (int e = tid; e < m * m; e += 1024) a[e] = double(it.A[e]);
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
    if (p != j && tid < m) {
      const double t = a[j + tid * m];
      a[j + tid * m] = a[p + tid * m];
      a[p + tid * m] = t;
    }
    __syncthreads();
    const double piv = a[j + j * m];
    if (tid < m) fcol[tid] = a[tid + j * m];
    __syncthreads();
    if (tid < m) a[j + tid * m] = (tid == j ? 1.0 : a[j + tid * m]) / piv;
    __syncthreads();
    for (int i = r; i < m; i += 64) {
      if (i == j) continue;
      const double f = fcol[i];
      for (int c = g; c < m; c += 16) a[i + c * m] = (c == j ? 0.0 : a[i + c * m]) - f * a[j + c * m];
    }
    __syncthreads();
  }
  for (int j = m - 1; j >= 0; --j) {
    const int p = perm[j];
    if (p != j && tid < m) {
      const double t = a[tid + j * m];
      a[tid + j * m] = a[tid + p * m];
      a[tid + p * m] = t;
    }
    __syncthreads();
  }
  for (int e = tid; e < m * m; e += 1024) it.Inv[e] = T(a[e]);
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
__global__ void add_kernel(const double* in, double* acc, int64_t ldacc, int64_t n, int64_t nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e % n, j = e / n;
    acc[i + j * ldacc] += in[e];
  }
}

// ---- right-hand-side blocks stored RHS-fastest: element (i, j) of an
// n x nrhs block at i nrhs + j
__global__ void gather_rm_kernel(const double* in, int64_t ld, const int64_t* idx, double* out, int64_t n,
                                 int64_t nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / nrhs, j = e - i * nrhs;
    out[e] = in[idx[i] + j * ld];
  }
}
__global__ void scatter_rm_kernel(const double* in, const int64_t* idx, double* out, int64_t ld, int64_t n,
                                  int64_t nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / nrhs, j = e - i * nrhs;
    out[idx[i] + j * ld] = in[e];
  }
}
// r = b - y; per block and column the sums of squares of r and of b (lanes
// run over the columns, 4 row groups per block, up to 512 columns)
__global__ __launch_bounds__(256) void residual_rm_kernel(const double* b, const double* y, double* r, int64_t n,
                                                          int64_t nrhs, int64_t rows, double* part) {
  __shared__ double red[2][4][512];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t r0 = blockIdx.x * rows, r1 = min(n, r0 + rows);
  double sr[8], sb[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) sr[q] = sb[q] = 0.0;
  for (int64_t i = r0 + ty; i < r1; i += 4) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t j = tx + 64 * q;
      if (j < nrhs) {
        const double bv = b[i * nrhs + j];
        const double rv = bv - y[i * nrhs + j];
        r[i * nrhs + j] = rv;
        sr[q] += rv * rv;
        sb[q] += bv * bv;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    red[0][ty][tx + 64 * q] = sr[q];
    red[1][ty][tx + 64 * q] = sb[q];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nrhs; j += 256) {
    part[blockIdx.x * 2 * nrhs + j] = red[0][0][j] + red[0][1][j] + red[0][2][j] + red[0][3][j];
    part[blockIdx.x * 2 * nrhs + nrhs + j] = red[1][0][j] + red[1][1][j] + red[1][2][j] + red[1][3][j];
  }
}
// nrm2[c] = sum over blocks of part[blk][c], in block order (deterministic)
__global__ void sum_parts_kernel(const double* part, int nblk, int64_t width, double* nrm2) {
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < width; c += int64_t(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int bk = 0; bk < nblk; ++bk) s += part[bk * width + c];
    nrm2[c] = s;
  }
}
// per block of rows and vector i: partial sums of V_i[r, j] w[r, j] (lanes
// over the columns, 4 row groups), written to part[blk][i][j]
__global__ __launch_bounds__(256) void multi_dot_kernel(const double* V, int64_t vstride, const double* w,
                                                        int64_t n, int64_t nrhs, int64_t rows, double* part) {
  __shared__ double red[4][512];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int i = blockIdx.y, cnt = gridDim.y;
  const double* v = V + int64_t(i) * vstride;
  const int64_t r0 = blockIdx.x * rows, r1 = min(n, r0 + rows);
  double s[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) s[q] = 0.0;
  for (int64_t r = r0 + ty; r < r1; r += 4) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t j = tx + 64 * q;
      if (j < nrhs) s[q] += v[r * nrhs + j] * w[r * nrhs + j];
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) red[ty][tx + 64 * q] = s[q];
  __syncthreads();
  const int64_t width = int64_t(cnt) * nrhs;
  for (int j = threadIdx.x; j < nrhs; j += 256)
    part[blockIdx.x * width + int64_t(i) * nrhs + j] = red[0][j] + red[1][j] + red[2][j] + red[3][j];
}
__global__ void multi_axpy_kernel(const double* V, int64_t vstride, int cnt, const double* coef, double sign,
                                  double* w, int64_t tot, int64_t nrhs) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = e % nrhs;
    double acc = 0.0;
    for (int i = 0; i < cnt; ++i) acc += coef[int64_t(i) * nrhs + j] * V[int64_t(i) * vstride + e];
    w[e] += sign * acc;
  }
}
__global__ void scale_cols_kernel(const double* w, const double* nrm2, double* v, int64_t tot, int64_t nrhs) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const double q = nrm2[e % nrhs];
    v[e] = q > 0.0 ? w[e] / sqrt(q) : 0.0;
  }
}
__global__ void scale_to_f_rm_kernel(const double* in, const double* cs, float* out, int64_t tot, int64_t nrhs) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x)
    out[e] = float(in[e] / cs[e % nrhs]);
}
__global__ void add_scaled_f_rm_kernel(const float* in, const double* cs, double* acc, int64_t tot, int64_t nrhs) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x)
    acc[e] += double(in[e]) * cs[e % nrhs];
}

template <class T>
__global__ __launch_bounds__(256) void copy_segments_kernel(const CopySeg* segs, const T* src, T* dst) {
  // one column per wave at a time, lanes along the rows (both sides contiguous)
  const CopySeg s = segs[blockIdx.y];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int c = blockIdx.x * 4 + wave; c < s.cols; c += gridDim.x * 4)
    for (int r = lane; r < s.rows; r += 64) dst[s.dst + int64_t(c) * s.rows + r] = src[s.src + int64_t(c) * s.src_ld + r];
}

// Copies a rows x cols column-major block (ld src_ld) into 16 x 16 tiles in
// the Schur kernel's lane order (rows = k, columns = the other index): tile
// (c, q) of the block at (q C + c) 256 elements, C = ceil(rows / 16)
// (column-outer, segment field pad = 0), or at (c Q + q) 256 elements,
// Q = ceil(cols / 16) (k-outer, pad = 1: rows of tiles follow k); inside a
// tile, element (k = 16 c + 4 g + s, column 16 q + r) at 4 (r + 16 g) + s.
// Places outside the block are written as zeros.  One work-group per block,
// threads along the tiled block (writes contiguous).
template <class T>
__global__ __launch_bounds__(256) void retile_kernel(const CopySeg* segs, const T* src, T* dst) {
  const CopySeg sg = segs[blockIdx.y];
  const int ck = (sg.rows + 15) >> 4, cq = (sg.cols + 15) >> 4;
  const int64_t len = int64_t(ck) * cq * 256;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < len; e += int64_t(gridDim.x) * blockDim.x) {
    const int t = int(e >> 8), p = int(e & 255);
    const int c = sg.pad ? t / cq : t % ck, q = sg.pad ? t % cq : t / ck;
    const int l = p >> 2, s4 = p & 3;
    const int k = 16 * c + 4 * (l >> 4) + s4, col = 16 * q + (l & 15);
    dst[sg.dst + e] = (k < sg.rows && col < sg.cols) ? src[sg.src + int64_t(col) * sg.src_ld + k] : T(0);
  }
}

// Sum of squares of a block in FP64, the same order in every kernel that
// calls it: thread t sums elements t, t + 256, ... then a tree over the
// work-group (256 threads).
template <class T>
__device__ __forceinline__ double block_sumsq(const T* p, int64_t len, double* red) {
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < len; e += 256) {
    const double v = double(p[e]);
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

template <class T>
__global__ __launch_bounds__(256) void block_sumsq_kernel(const BlockRef* blocks, const T* S, double* out) {
  __shared__ double red[256];
  const BlockRef b = blocks[blockIdx.x];
  const double s = block_sumsq(S + b.off, b.len, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

template <class T>
__global__ __launch_bounds__(256) void drop_small_kernel(const DropItem* items, T* S, uint8_t* flag) {
  __shared__ double red[256];
  const DropItem it = items[blockIdx.x];
  const double sq = block_sumsq(S + it.off, it.len, red);  // the same value in every thread
  const bool drop = sq < it.thr2;
  if (drop)
    for (int64_t e = threadIdx.x; e < it.len; e += 256) S[it.off + e] = T(0);
  if (threadIdx.x == 0) flag[it.idx] = drop ? (sq > 0.0 ? 1 : 2) : 0;
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
  switch (g.role) {
    case ROLE_FACTOR: return launch_gemm_factor<T>(g, st);
    case ROLE_SOLVE: return launch_gemm_solve<T>(g, st);
    case ROLE_MATVEC:
      if constexpr (sizeof(T) == 8) return launch_gemm_matvec(g, st);
      return;
    default:
      if (g.amode == 2) return launch_gemm_transform_gen<T>(g, st);
      return launch_gemm_transform<T>(g, st);
  }
}
template void launch_gemm<double>(const GemmLaunch&, hipStream_t);
template void launch_gemm<float>(const GemmLaunch&, hipStream_t);

template <class T>
void launch_schur(const SchurLaunch& g, int cls, hipStream_t st) {
  if (g.ntiles <= 0) return;
  if constexpr (sizeof(T) == 4) {
    if (cls == 1) {
      hipLaunchKernelGGL((schur_kernel<T, 1>), dim3(g.ntiles), dim3(64), 0, st, g);
      return;
    }
    if (cls == 2) {
      hipLaunchKernelGGL((schur_kernel<T, 2>), dim3(g.ntiles), dim3(64), 0, st, g);
      return;
    }
  }
  hipLaunchKernelGGL((schur_kernel<T, 0>), dim3(g.ntiles), dim3(64), 0, st, g);
}
template void launch_schur<double>(const SchurLaunch&, int, hipStream_t);
template void launch_schur<float>(const SchurLaunch&, int, hipStream_t);

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
  hipLaunchKernelGGL(inverse_kernel<T>, dim3(count), dim3(1024), 0, st, items, flag);
}
template void launch_inverse<double>(const InvItem<double>*, int, int*, hipStream_t);
template void launch_inverse<float>(const InvItem<float>*, int, int*, hipStream_t);

template <class T>
void launch_copy_segments(const CopySeg* segs, int count, const T* src, T* dst, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int c = (count - c0) < 65535 ? (count - c0) : 65535;
    hipLaunchKernelGGL(copy_segments_kernel<T>, dim3(8, c), dim3(256), 0, st, segs + c0, src, dst);
  }
}
template <class T>
void launch_block_sumsq(const BlockRef* blocks, int count, const T* S, double* out, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += 1 << 30) {
    const int c = count - c0 < (1 << 30) ? count - c0 : (1 << 30);
    hipLaunchKernelGGL(block_sumsq_kernel<T>, dim3(c), dim3(256), 0, st, blocks + c0, S, out + c0);
  }
}
template void launch_block_sumsq<double>(const BlockRef*, int, const double*, double*, hipStream_t);
template void launch_block_sumsq<float>(const BlockRef*, int, const float*, double*, hipStream_t);
template <class T>
void launch_drop_small(const DropItem* items, int count, T* S, uint8_t* flag, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(drop_small_kernel<T>, dim3(count), dim3(256), 0, st, items, S, flag);
}
template void launch_drop_small<double>(const DropItem*, int, double*, uint8_t*, hipStream_t);
template void launch_drop_small<float>(const DropItem*, int, float*, uint8_t*, hipStream_t);

template <class T>
void launch_retile(const CopySeg* segs, int count, const T* src, T* dst, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int c = (count - c0) < 65535 ? (count - c0) : 65535;
    hipLaunchKernelGGL(retile_kernel<T>, dim3(4, c), dim3(256), 0, st, segs + c0, src, dst);
  }
}
template void launch_retile<double>(const CopySeg*, int, const double*, double*, hipStream_t);
template void launch_retile<float>(const CopySeg*, int, const float*, float*, hipStream_t);
template void launch_copy_segments<double>(const CopySeg*, int, const double*, double*, hipStream_t);
template void launch_copy_segments<float>(const CopySeg*, int, const float*, float*, hipStream_t);

void launch_gather_rm(const double* in, int64_t ld, const int64_t* idx, double* out, int64_t n, int64_t nrhs,
                      hipStream_t st) {
  if (n * nrhs > 0) hipLaunchKernelGGL(gather_rm_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, ld, idx, out, n, nrhs);
}
void launch_scatter_rm(const double* in, const int64_t* idx, double* out, int64_t ld, int64_t n, int64_t nrhs,
                       hipStream_t st) {
  if (n * nrhs > 0) hipLaunchKernelGGL(scatter_rm_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, idx, out, ld, n, nrhs);
}
int residual_rm_blocks(int64_t n) {
  int64_t b = (n + 63) / 64;
  return int(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}
void launch_residual_rm(const double* b, const double* y, double* r, int64_t n, int64_t nrhs, double* part,
                        double* nrm2, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return;
  const int nblk = residual_rm_blocks(n);
  const int64_t rows = (n + nblk - 1) / nblk;
  hipLaunchKernelGGL(residual_rm_kernel, dim3(nblk), dim3(256), 0, st, b, y, r, n, nrhs, rows, part);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(grid_for(2 * nrhs)), dim3(256), 0, st, part, nblk, 2 * nrhs, nrm2);
}
void launch_multi_dot(const double* V, int64_t vstride, int cnt, const double* w, int64_t n, int64_t nrhs,
                      double* part, double* out, hipStream_t st) {
  if (n <= 0 || nrhs <= 0 || cnt <= 0) return;
  const int nblk = residual_rm_blocks(n);
  const int64_t rows = (n + nblk - 1) / nblk;
  hipLaunchKernelGGL(multi_dot_kernel, dim3(nblk, cnt), dim3(256), 0, st, V, vstride, w, n, nrhs, rows, part);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(grid_for(int64_t(cnt) * nrhs)), dim3(256), 0, st, part, nblk,
                     int64_t(cnt) * nrhs, out);
}
void launch_multi_axpy(const double* V, int64_t vstride, int cnt, const double* coef, double sign, double* w,
                       int64_t n, int64_t nrhs, hipStream_t st) {
  if (n * nrhs > 0 && cnt > 0)
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, V, vstride, cnt, coef, sign, w,
                       n * nrhs, nrhs);
}
void launch_scale_cols(const double* w, const double* nrm2, double* v, int64_t n, int64_t nrhs, hipStream_t st) {
  if (n * nrhs > 0)
    hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, w, nrm2, v, n * nrhs, nrhs);
}
void launch_scale_to_f_rm(const double* in, const double* cs, float* out, int64_t n, int64_t nrhs, hipStream_t st) {
  if (n * nrhs > 0) hipLaunchKernelGGL(scale_to_f_rm_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, cs, out, n * nrhs, nrhs);
}
void launch_add_scaled_f_rm(const float* in, const double* cs, double* acc, int64_t n, int64_t nrhs, hipStream_t st) {
  if (n * nrhs > 0)
    hipLaunchKernelGGL(add_scaled_f_rm_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, cs, acc, n * nrhs, nrhs);
}

// One work-group per block, threads along the block's elements (k fastest).
// The value is formed exactly as gen4 forms a generated B element.
__global__ __launch_bounds__(256) void kernel_blocks_kernel(const KernelBlock* blocks, const double* x, int dim,
                                                          int kern, double scale, double diag, double param,
                                                          double* out) {
  const KernelBlock b = blocks[blockIdx.x];
  const int64_t len = int64_t(b.nt) * b.ns;
  const double* pr = x + int64_t(b.t0) * dim;
  const double* pc = x + int64_t(b.s0) * dim;
  for (int64_t e = threadIdx.x; e < len; e += blockDim.x) {
    const int k = int(e % b.ns), j = int(e / b.ns);
    double val;
    if (b.diag_blk && j == k) {
      val = diag;
    } else {
      double d2 = 0.0;
      for (int a = 0; a < dim; ++a) {
        const double d = pr[j * dim + a] - pc[k * dim + a];
        d2 += d * d;
      }
      val = kern == 0   ? kernel_value<0>(d2, scale, param)
            : kern == 1 ? kernel_value<1>(d2, scale, param)
                        : kernel_value<2>(d2, scale, param);
    }
    out[b.off + e] = val;
  }
}

void launch_kernel_blocks(const KernelBlock* blocks, int count, const double* x, int dim, int kern,
                          double scale, double diag, double param, double* out, hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(kernel_blocks_kernel, dim3(count), dim3(256), 0, st, blocks, x, dim, kern, scale, diag, param,
                       out);
}

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
void launch_add(const double* in, double* acc, int64_t ldacc, int64_t n, int64_t nrhs, hipStream_t st) {
  if (n * nrhs > 0) hipLaunchKernelGGL(add_kernel, dim3(grid_for(n * nrhs)), dim3(256), 0, st, in, acc, ldacc, n, nrhs);
}

}  // namespace h2
