// Device kernels of libh2sp and their work-item descriptors.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2 {

// One K-segment of a batched GEMM item: acc += op(A) (M x K) * op(B) (K x N).
// opA = 0: A column-major M x K (element (i, k) at A[i + k lda]);
// opA = 1: A stored K x M   (element (i, k) at A[k + i lda]).
// opB = 0: B column-major K x N; opB = 1: B stored N x K.
// gen = 1: A is generated, A(i, k) = kernel(pr_i, pc_k) with pr = (const
// double*) A and pc the points along K (dim-strided); gen = 2: B is generated
// the same way, B(k, j) = kernel(pr_j, pc_k) with pr = (const double*) B
// (the kernel is symmetric).  kernel(x, y) = scale / |x - y| (gkern 0),
// scale exp(-|x - y|^2) (gkern 1), or with r = |x - y| scale r / d below d and
// scale d / r from d on (gkern 2, d = gparam).  diag = 1 puts the diagonal value where the two
// indices are equal (a cluster against itself).  scale, the diagonal value
// and dim belong to the item (so that items of different matrices can share
// a launch).
struct GemmSeg {
  const void* A;
  const void* B;
  const double* pc;
  int32_t K, lda, ldb;
  uint8_t opA, opB, gen, diag;
};

// Output of a batched GEMM item (M x N), split into quadrants at row rs and
// column cs: q0 = [0,rs) x [0,cs), q1 = [0,rs) x [cs,N), q2 = [rs,M) x [0,cs),
// q3 = [rs,M) x [cs,N).  Destination q (0..3) receives its quadrant with local
// indices; destination 4 receives quadrant 0 again.  trans[q] = 1 stores the
// transpose (element (i, j) at out[j + i ld]).  A null out drops the quadrant.
struct GemmItem {
  int32_t M, N, seg_begin, seg_end;
  int32_t rs, cs;
  void* out[5];
  int32_t ld[5];
  uint8_t trans[5];
  uint8_t gkern;           // generated operands: 0 inverse distance, 1 exp(-r^2), 2 r/d | d/r
  uint8_t store;           // 1: store the sum (a partial sum of a split item), whatever the launch's mode
  int32_t gdim;            // generated operands: point dimension
  double gscale, gdiag;    // generated operands: kernel scale, diagonal value
  double gparam;           // generated operands: d of kernel 2
};

enum GemmMode { GEMM_STORE = 0, GEMM_ADD = 1, GEMM_SUB = 2 };
// The same kernel is instantiated once per role so that profiles separate the
// sparsification transforms, the factorisation, the solve sweeps and the matvec.
enum GemmRole { ROLE_TRANSFORM = 0, ROLE_FACTOR = 1, ROLE_SOLVE = 2, ROLE_MATVEC = 3 };

// Operand layout codes of a launch: amode 0 = A K-contiguous (opA = 1),
// 1 = A M-contiguous (opA = 0), 2 = A generated; bmode 0 = B K-contiguous
// (opB = 0), 1 = B N-contiguous (opB = 1), 2 = B generated.  All segments of
// a launch share them.
struct GemmLaunch {
  int amode, bmode;
  const GemmItem* items;
  const GemmSeg* segs;
  const int32_t* tiles;   // per work-group: (item << 8) | (tile_row << 4) | tile_col
  int32_t ntiles;
  int mode;
  int role;
  int kern;               // kernel of generated operands (GemmItem::gkern of every item)
  int variant;            // output tile shape (gemm_shape)
  int wg_rows;            // waves per work-group: the row tiles of one tile column (solve sweeps), else 1
};

// Output tile shapes the GEMM kernel is built with, per role and operand
// layout pair: variant v in precision prec (0 FP64, 1 FP32) is a tile of
// ((code >> 4) & 15) x (code & 15) blocks of 16 x 16 (rows x columns) per wave,
// run by the LDS-staged kernel when code has kGemmLds, code 0 when
// that variant is not built.  Variant 0 is the default; the tuning table
// selects another per precision, role, layout and row bucket.  Measured
// defaults: on short-K work (the solve sweeps, the pivot GEMMs, the transforms
// with M-contiguous operands) 32 x 32 tiles, with more waves per SIMD, beat
// 64 x 64; a generated operand is shared by more blocks in 64 x 32 tiles, and
// the transforms whose two operands both run along K take 64 x 32 too.  The
// solve sweeps also build the LDS-staged kernel, whose work-group stages each
// 16-wide k step of the right-hand sides and of the S block once for all its
// waves.  FP64
// variants keep at most 16 blocks (the accumulators take twice the
// registers), 8 in the solve sweeps, whose kernel holds two chunks of
// operands.
constexpr int kGemmVariants = 6;
constexpr int kSolveWaves = 4;  // most waves (row tiles) per work-group of the solve sweeps
constexpr int kGemmLds = 0x100; // shape flag: the solve kernel that stages operand chunks in LDS
constexpr int gemm_pick(int v, int a, int b, int c, int d, int e = 0, int f = 0) {
  return v == 0 ? a : v == 1 ? b : v == 2 ? c : v == 3 ? d : v == 4 ? e : v == 5 ? f : 0;
}
constexpr int gemm_shape(int prec, int role, int am, int bm, int v) {
  const int m = am * 3 + bm;
  int code = 0;
  switch (role) {
    case ROLE_TRANSFORM:
      code = (m == 0 || m == 6 || m == 7) ? gemm_pick(v, 0x42, 0x22, 0x44, 0)
             : (m == 3)                   ? gemm_pick(v, 0x22, 0x42, 0x44, 0)
                                          : 0;
      break;
    case ROLE_FACTOR: code = m == 0 ? gemm_pick(v, 0x22, 0x42, 0x44, 0) : 0; break;
    case ROLE_SOLVE:
      code = (m == 3 || m == 4) ? gemm_pick(v, 0x22, 0x42, 0x24, 0x44, kGemmLds | 0x22, kGemmLds | 0x24) : 0;
      if (prec == 0 && (code & kGemmLds)) code = 0;  // the LDS-staged kernel is FP32 only
      break;
    case ROLE_MATVEC:
      code = (m == 3 || m == 4) ? gemm_pick(v, 0x44, 0x42, 0x22, 0)
             : m == 5           ? gemm_pick(v, 0x42, 0x22, 0x44, 0x81)
                                : 0;
      break;
    default: code = 0;
  }
  if (prec == 0 && ((code >> 4) & 15) * (code & 15) > (role == ROLE_SOLVE ? 8 : 16)) code = 0;
  return code;
}
// whether a role's kernels are built for a layout pair
constexpr bool gemm_layout_supported(int role, int amode, int bmode) {
  return gemm_shape(1, role, amode, bmode, 0) != 0;
}

template <class T>
void launch_gemm(const GemmLaunch& g, hipStream_t st);
// the launches of one role (one translation unit each)
template <class T>
void launch_gemm_transform(const GemmLaunch& g, hipStream_t st);
template <class T>
void launch_gemm_transform_gen(const GemmLaunch& g, hipStream_t st);
template <class T>
void launch_gemm_factor(const GemmLaunch& g, hipStream_t st);
template <class T>
void launch_gemm_solve(const GemmLaunch& g, hipStream_t st);
void launch_gemm_matvec(const GemmLaunch& g, hipStream_t st);  // FP64 only

// Compact work list of the Schur update S_ij -= Z_ki^T S_kj (offsets in
// elements into S and into the buffer of Z_ki blocks; every operand has leading
// dimension equal to its row count).  Tiles: (item << 8) | (tile_row << 4) |
// tile_col, schur_edge<T> x schur_edge<T> tiles: 128 in FP32, so that a target
// of up to 128 x 128 (every pivot block and S block of the library: clusters
// have at most 128 rows) is one tile whose operands cross the memory system
// once per chunk, and 64 in FP64, whose accumulators take twice the registers.
// A target with a long K is split into parts: part 0 subtracts its sum from S
// directly, every further part stores its sum (M x N, ld M) in the partial
// buffer and a reduction item subtracts those sums, in a fixed order.
// The kernel reads every operand through a buffer resource of the block's own
// size, so it reads nothing outside the blocks the descriptors name.
template <class T>
constexpr int schur_edge = sizeof(T) == 4 ? 128 : 64;
struct SchurItem {
  int64_t out_off;   // into S (partial == 0) or the partial buffer (partial == 1)
  int32_t M, N, seg_begin, seg_end;
  int32_t partial, ksum;  // ksum: K summed over the item's segments (planning)
};
struct SchurSeg {
  int64_t b_off;     // S_kj (K x N) in the launch's S operand array: in tiles or in place (ld K)
  int32_t a_off, K;  // Z_ki (K x M) in tiles (see launch_retile) in the Z tile buffer
};
struct SchurReduce {
  int64_t s_off, p_off;  // target in S; first of `parts` consecutive M x N partial sums
  int32_t len, parts;    // len = M N
};
struct SchurLaunch {
  const SchurItem* items;
  const SchurSeg* segs;
  const int32_t* tiles;
  int32_t ntiles;
  void* S;               // targets (in place, column-major)
  const void* Sb;        // S_kj operands: tiled copies (tiled_b = 1) or S itself (tiled_b = 0)
  const void* Z;         // Z_ki operands, in tiles
  void* P;               // partial buffer
  int32_t tiled_b;
  int32_t kouter;        // tile layout of Z and the tiled S_kj (see launch_retile): 1 k-outer, 0 column-outer
};
// Tile class (each class has a kernel of its own, with the register budget
// of its shapes; see schur_kernel): 0 when the tile has at most 4 blocks of
// 16 along both sides (every FP64 tile), 1 when the longer side has 5, 2 when
// it has 6 to 8.
constexpr int kSchurClasses = 3;
template <class T>
constexpr int schur_tile_class(int M, int N, int m0, int n0, int edge = schur_edge<T>) {
  const int e = M - m0 > N - n0 ? M - m0 : N - n0;
  const int b = (e < edge ? e : edge) + 15;
  return b / 16 <= 4 ? 0 : b / 16 == 5 ? 1 : 2;
}
// Tile code of the Schur kernels: (item << 8) | (row << 4) | column in tiles
// of the full edge, or with row and column + 8 in tiles of half the edge (a
// target of class 2 cut into tiles of class 0, when the tuning table asks:
// more waves per SIMD for the same work, at twice the operand reads).
inline int32_t schur_tile_code(uint32_t item, int a, int b, bool half) {
  return int32_t((item << 8) | ((half ? a + 8 : a) << 4) | (half ? b + 8 : b));
}
template <class T>
void launch_schur(const SchurLaunch& g, int cls, hipStream_t st);
template <class T>
void launch_schur_reduce(const SchurReduce* items, int count, const T* P, T* S, hipStream_t st);

// Householder QR of one cluster basis B (n x r, column-major, ld n), n <= 128,
// r <= 64.  Writes the explicit square Q (n x n, ld n) and R^ = rows 0..k-1 of
// R (k x r, ld k).  k = 0: Q = I and nothing else.
struct QrItem {
  const double* B;
  double* Q;
  double* Rhat;
  int32_t n, r, k, pad;
};
void launch_qr(const QrItem* items, int count, hipStream_t st);

// Inverse of a pivot block (m x m, column-major, m <= 128) computed in FP64 by
// Gauss-Jordan elimination with partial pivoting; a zero pivot sets *flag = 1.
template <class T>
struct InvItem {
  const T* A;
  T* Inv;
  int32_t m, pad;
};
template <class T>
void launch_inverse(const InvItem<T>* items, int count, int* flag, hipStream_t st);

// Block threshold ILU (drop tolerance): sums of squares of blocks of S and
// the drop of small fill blocks.  Both reduce in FP64 in a fixed order (per
// thread strided partial sums, then a tree over the work-group).
struct BlockRef {
  int64_t off;  // first element in S
  int64_t len;  // elements
};
template <class T>
void launch_block_sumsq(const BlockRef* blocks, int count, const T* S, double* out, hipStream_t st);
// For every item: if the block's sum of squares is below thr2 the block is
// set to zero and flag[idx] to 1, or to 2 when it was zero already (a fill
// block that no update reached); else flag[idx] = 0.
struct DropItem {
  int64_t off;
  double thr2;
  int32_t len, idx;
};
template <class T>
void launch_drop_small(const DropItem* items, int count, T* S, uint8_t* flag, hipStream_t st);

// Copies a rows x cols block from src (leading dimension src_ld) to a
// contiguous block of dst (leading dimension rows), for every segment.
struct CopySeg {
  int64_t dst, src;          // dst: rows x cols, ld rows; src: ld src_ld
  int32_t rows, cols, src_ld, pad;  // pad: launch_retile's layout (1 k-outer, 0 column-outer)
};
template <class T>
void launch_copy_segments(const CopySeg* segs, int count, const T* src, T* dst, hipStream_t st);
// For every segment: dst + dst_off receives the transpose (cols x rows,
// column-major) of the rows x cols column-major block at src + src_off
// (src_ld = rows).  LDS tiles of 32 x 32, reads and writes both contiguous.
template <class T>
void launch_transpose_blocks(const CopySeg* segs, int count, const T* src, T* dst, hipStream_t st);
// For every segment: the rows x cols block at src (leading dimension src_ld)
// into 16 x 16 tiles at dst, in the order the Schur kernel's lanes read them:
// tile (c, q) at dst + (q C + c) 256 with C = ceil(rows / 16), element
// (16 c + 4 g + s, 16 q + r) at 4 (r + 16 g) + s inside it; the padding to
// whole tiles is zero.  dst needs C ceil(cols / 16) 256 elements.
template <class T>
void launch_retile(const CopySeg* segs, int count, const T* src, T* dst, hipStream_t st);

// Kernel blocks written out: element (k, j) of block b, at out[b.off + k + j ns],
// is kernel(x_{t0 + j}, x_{s0 + k}) of kind kern (as GemmItem::gkern; dim coordinates per point, points
// consecutive in x), or diag where diag_blk is set and t0 + j == s0 + k.  The
// values are bit for bit those the GEMM kernels generate for a B operand of
// the same block (gen = 2).
struct KernelBlock {
  int64_t off;
  int32_t t0, s0, nt, ns;
  int32_t diag_blk, pad;
};
void launch_kernel_blocks(const KernelBlock* blocks, int count, const double* x, int dim, int kern,
                          double scale, double diag, double param, double* out, hipStream_t st);

// Scratch of the entry point that allocates nothing (h2_apply_inverse_noalloc):
// one static device array of kNoAllocScratchBytes per GPU, held until the
// process ends.  noalloc_scratch gives its device address on the current
// device (taken once per device with hipGetSymbolAddress).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch(void** ptr);

// Small element-wise helpers.
void launch_fill(double* p, int64_t n, double v, hipStream_t st);
void launch_fill_f(float* p, int64_t n, float v, hipStream_t st);
void launch_fill_i(int* p, int64_t n, int v, hipStream_t st);
void launch_cast_d2f(const double* in, float* out, int64_t n, hipStream_t st);
void launch_add(const double* in, double* acc, int64_t ldacc, int64_t n, int64_t nrhs,
                hipStream_t st);

// Right-hand-side blocks inside the solve and the matvec are stored
// RHS-fastest: element (i, j) of an n x nrhs block at i nrhs + j.
// out[i nrhs + j] = in[idx[i] + j ld]  (caller's column-major block, rows picked by idx)
void launch_gather_rm(const double* in, int64_t ld, const int64_t* idx, double* out, int64_t n, int64_t nrhs,
                      hipStream_t st);
// out[idx[i] + j ld] = in[i nrhs + j]
void launch_scatter_rm(const double* in, const int64_t* idx, double* out, int64_t ld, int64_t n, int64_t nrhs,
                       hipStream_t st);
// r = b - y, then nrm2[j] = sum_i r_ij^2 and nrm2[nrhs + j] = sum_i b_ij^2 in a
// fixed order; part: scratch of residual_rm_blocks(n) * 2 * nrhs doubles;
// nrhs <= 512
int residual_rm_blocks(int64_t n);
void launch_residual_rm(const double* b, const double* y, double* r, int64_t n, int64_t nrhs, double* part,
                        double* nrm2, hipStream_t st);
// Krylov helpers on RHS-fastest blocks (n x nrhs, nrhs <= 512); vector i of
// a set starts at V + i vstride.  All sums run in a fixed order.
// out[i nrhs + j] = sum_r V_i[r, j] w[r, j] for i < cnt; part: scratch of
// residual_rm_blocks(n) * cnt * nrhs doubles
void launch_multi_dot(const double* V, int64_t vstride, int cnt, const double* w, int64_t n, int64_t nrhs,
                      double* part, double* out, hipStream_t st);
// w[r, j] += sign * sum_{i < cnt, in order} coef[i nrhs + j] V_i[r, j]
void launch_multi_axpy(const double* V, int64_t vstride, int cnt, const double* coef, double sign, double* w,
                       int64_t n, int64_t nrhs, hipStream_t st);
// v[r, j] = w[r, j] / sqrt(nrm2[j]), or 0 where nrm2[j] is 0
void launch_scale_cols(const double* w, const double* nrm2, double* v, int64_t n, int64_t nrhs, hipStream_t st);
// float out = in / colscale[j];  double acc += float in * colscale[j]
void launch_scale_to_f_rm(const double* in, const double* cs, float* out, int64_t n, int64_t nrhs, hipStream_t st);
void launch_add_scaled_f_rm(const float* in, const double* cs, double* acc, int64_t n, int64_t nrhs, hipStream_t st);

}  // namespace h2
