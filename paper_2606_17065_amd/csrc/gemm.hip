// Grouped expert GEMMs over uneven per-expert row counts, for gfx950.
//
//   GEMM 1 (SwiGLU):  h = silu(Xp W1_e^T) * (Xp W3_e^T)     [rows of e, f]
//   GEMM 2:           Y = h W2_e^T                           [rows of e, d]
//
// Both products are "NT": the A rows (tokens) and the B rows (weight rows)
// are contiguous along K, which is exactly the operand layout of the MFMA
// fragments.  A tile scheduler maps blockIdx.x to (expert, row tile) from
// the exclusive scan of ceil(rows_e / BM); blocks past the last tile exit.
#include "common.h"
#include "internal.h"

namespace moe_gemm {

__device__ __forceinline__ float silu(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// tile_start[e] = sum_{e' < e} ceil(rows_e' / BM); tile_start[E] = total.
__global__ __launch_bounds__(1024) void ffn_tiles(const int32_t* __restrict__ offsets, int E,
                                                  int BM, int32_t* __restrict__ tile_start) {
  __shared__ int buf[2][MOE_MAX_E + 1];
  const int e = threadIdx.x;
  int v = 0;
  if (e < E) v = (offsets[e + 1] - offsets[e] + BM - 1) / BM;
  buf[0][e] = v;
  __syncthreads();
  int cur = 0;
  for (int off = 1; off < 1024; off <<= 1) {
    int x = buf[cur][e];
    if (e >= off) x += buf[cur][e - off];
    buf[cur ^ 1][e] = x;
    cur ^= 1;
    __syncthreads();
  }
  // buf[cur][e] = inclusive sum
  if (e < E) tile_start[e + 1] = buf[cur][e];
  if (e == 0) tile_start[0] = 0;
}

__device__ __forceinline__ bool find_tile(const int32_t* __restrict__ tile_start,
                                          const int32_t* __restrict__ offsets, int E, int BM,
                                          int N, int mt, int& e_out, int& row0, int& rows) {
  if (mt >= tile_start[E]) return false;
  int lo = 0, hi = E - 1;  // largest e with tile_start[e] <= mt
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= mt) lo = mid;
    else hi = mid - 1;
  }
  e_out = lo;
  row0 = offsets[lo] + (mt - tile_start[lo]) * BM;
  rows = min(BM, offsets[lo + 1] - row0);
  // rows outside [0, N) are never touched, whatever the offsets hold
  if (row0 < 0 || row0 >= N) return false;
  rows = min(rows, N - row0);
  return rows > 0;
}

// Logical tile order of the 256-row kernels: expert by expert; inside an
// expert, groups of NG column tiles, and inside a group row tile by row
// tile with the NG column tiles of a row tile adjacent.  A run of
// consecutive tiles (what one XCD's CUs hold at once) then covers all row
// tiles of an expert against a few weight slices, so both operands are
// re-read from that XCD's L2 rather than from HBM.
constexpr int NG = 4;

__device__ __forceinline__ bool find_tile_grouped(const int32_t* __restrict__ tile_start,
                                                  const int32_t* __restrict__ offsets, int E,
                                                  int BMr, int N, int n_tiles, int Lt, int& e_out,
                                                  int& row0, int& rows, int& nt) {
  if (Lt >= tile_start[E] * n_tiles) return false;
  int lo = 0, hi = E - 1;  // largest e with tile_start[e] * n_tiles <= Lt
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] * n_tiles <= Lt) lo = mid;
    else hi = mid - 1;
  }
  const int mc = tile_start[lo + 1] - tile_start[lo];
  const int local = Lt - tile_start[lo] * n_tiles;
  const int g = local / (mc * NG);
  const int rem = local - g * mc * NG;
  const int ng = min(NG, n_tiles - g * NG);
  const int mt = rem / ng;
  nt = g * NG + (rem - mt * ng);
  e_out = lo;
  row0 = offsets[lo] + mt * BMr;
  rows = min(BMr, offsets[lo + 1] - row0);
  if (row0 < 0 || row0 >= N) return false;
  rows = min(rows, N - row0);
  return rows > 0;
}

// Logical tile of block b: XCD b % 8 takes the b / 8-th tile of its run of
// ceil(tiles / 8) consecutive tiles, so the 8 XCDs get equal shares of the
// tiles that exist however far the grid (sized for the worst-case routing)
// exceeds them.  Blocks past the end get an index find_tile_grouped rejects.
__device__ __forceinline__ int xcd_tile(const int32_t* __restrict__ tile_start, int E,
                                        int n_tiles, int grid_total, int b) {
  const int per = min((tile_start[E] * n_tiles + 7) >> 3, grid_total >> 3);
  const int j = b >> 3;
  return j < per ? (b & 7) * per + j : 0x7fffffff;
}

// ------------------------------------------------------- BF16 MFMA, 256x128
// Macro tile 256 token rows x 128 weight rows, 4 wavefronts (2 x 2) each
// owning 128 x 64 as 4 x 2 tiles of v_mfma_f32_32x32x16_bf16; two blocks
// share a CU (LDS and registers are sized for it), so one block's
// prologue, barriers and epilogue overlap the other's MFMA work.
// Operands move HBM -> LDS with gfx950's direct-to-LDS loads
// (global_load_lds_dwordx4: a wavefront instruction deposits 64 x 16 bytes
// contiguously) through a ring of three K-steps of 32; no VGPRs are spent
// on staging.  A stage holds 64 bytes per row; the 16-byte chunk c of row R
// sits at position c ^ swz(R), which keeps the fragment reads of 8- and of
// 16-lane groups on distinct LDS banks.  A lane loads the global chunk that
// belongs at its fixed LDS slot.
// The MFMA takes the weight fragment as its first operand, so each lane
// ends up holding one token row and runs of 4 consecutive output columns;
// the epilogue stages the tile through LDS and writes 16-byte row segments.
// SwiGLU mode: weight rows 0..63 are W1 rows n0..n0+63, 64..127 the
// matching W3 rows; a wavefront's column tiles 0 and 1 are the two halves
// of the same 32 outputs.  Rows of a partial row tile load a clamped
// (valid) row; their results are never stored.
// Blocks are remapped so that each XCD (the hardware deals blocks to the 8
// XCDs round-robin) walks a contiguous run of the grouped tile order; the
// runs split the tiles that exist (counted on the device), not the grid,
// which is sized for the worst case of the routing.

constexpr int GBM = 256, GBN = 128, GBK = 32, NSTAGE = 3;
constexpr int STAGE_A = GBM * GBK * 2;   // bytes of the token operand in a stage
constexpr int STAGE_B = GBN * GBK * 2;   // bytes of the weight operand
constexpr int STAGE_BYTES = STAGE_A + STAGE_B;
constexpr int EPI_BYTES = GBM * (128 + 8) * 2;
constexpr int DMA_LDS = NSTAGE * STAGE_BYTES > EPI_BYTES ? NSTAGE * STAGE_BYTES : EPI_BYTES;
constexpr int A_INS = GBM / 4 / 16;      // DMA instructions per wavefront per stage
constexpr int B_INS = GBN / 4 / 16;
constexpr int VM_PER_STAGE = A_INS + B_INS;

__device__ __forceinline__ int swz(int R) { return ((R >> 1) ^ (R >> 2)) & 3; }

// s_waitcnt vmcnt(n) lgkmcnt(0) (gfx9 encoding: vmcnt[3:0] in bits 3:0,
// vmcnt[5:4] in bits 15:14, expcnt in 6:4 left at its maximum, lgkmcnt in
// 11:8 = 0).
#define WAIT_VM_LGKM0(n) __builtin_amdgcn_s_waitcnt((((n) & 15) | (((n) >> 4) << 14)) | (7 << 4))

// Workgroup barrier without the release fence of __syncthreads (which would
// wait for every outstanding direct-to-LDS load); the inline-asm memory
// clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void stage_barrier() {
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// The pipelined main loop shared by every 256x128 kernel.  Each lane
// brings its DMA source pointers (one per 16-row instruction, already at
// its K-chunk); the loop adds kstep*32 elements to them.
template <int AI, int BI>
__device__ __forceinline__ void mma_pipeline(char* lds, const bf16_t* (&asrc)[AI],
                                             const bf16_t* (&bsrc)[BI], int nk, int wv,
                                             int lane, const int (&aoff)[4], const int (&asw)[4],
                                             const int (&boff)[2], const int (&bsw)[2],
                                             f32x16 (&acc)[4][2]) {
  typedef __attribute__((address_space(3))) void lds_void;
  constexpr int VMS = AI + BI;
  const int fh = lane >> 5;
#define ISSUE(kstep)                                                                           \
  {                                                                                            \
    char* st_ = lds + ((kstep) % NSTAGE) * STAGE_BYTES;                                        \
    const int k0_ = (kstep) * GBK;                                                             \
    _Pragma("unroll") for (int i = 0; i < AI; ++i) __builtin_amdgcn_global_load_lds(           \
        asrc[i] + k0_, (lds_void*)(st_ + (wv * (GBM / 4) + i * 16) * 64), 16, 0, 0);           \
    _Pragma("unroll") for (int i = 0; i < BI; ++i) __builtin_amdgcn_global_load_lds(           \
        bsrc[i] + k0_, (lds_void*)(st_ + STAGE_A + (wv * (GBN / 4) + i * 16) * 64), 16, 0, 0); \
  }
#define READ_FRAGS(AF, BF, stp, ks)                                                      \
  {                                                                                      \
    const char* st_ = lds + ((stp) % NSTAGE) * STAGE_BYTES;                              \
    const int c_ = (ks) * 2 + fh;                                                        \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) AF[i] =                                \
        *(const bf16x8*)(st_ + aoff[i] + ((c_ ^ asw[i]) << 4));                          \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) BF[j] =                                \
        *(const bf16x8*)(st_ + boff[j] + ((c_ ^ bsw[j]) << 4));                          \
  }
#define MFMA8(AF, BF)                                                                    \
  _Pragma("unroll") for (int i = 0; i < 4; ++i) _Pragma("unroll") for (int j = 0; j < 2; \
                                                                       ++j) acc[i][j] =  \
      __builtin_amdgcn_mfma_f32_32x32x16_bf16(BF[j], AF[i], acc[i][j], 0, 0, 0);
  if (nk <= 0) return;
  bf16x8 a0[4], b0[2], a1[4], b1[2];
  ISSUE(0);
  if (nk > 1) ISSUE(1);
  if (nk > 2) ISSUE(2);
  if (nk > 2) {
    WAIT_VM_LGKM0(2 * VMS);
  } else if (nk > 1) {
    WAIT_VM_LGKM0(VMS);
  } else {
    WAIT_VM_LGKM0(0);
  }
  stage_barrier();
  READ_FRAGS(a0, b0, 0, 0);
  for (int kt = 0; kt + 1 < nk; ++kt) {
    __builtin_amdgcn_iglp_opt(1);
    READ_FRAGS(a1, b1, kt, 1);
    MFMA8(a0, b0);
    // step kt+1 must have landed: at most step kt+2 remains in flight
    if (kt + 2 < nk) {
      WAIT_VM_LGKM0(VMS);
    } else {
      WAIT_VM_LGKM0(0);
    }
    stage_barrier();  // every wavefront's reads of stage kt are done
    if (kt + 3 < nk) ISSUE(kt + 3);
    READ_FRAGS(a0, b0, kt + 1, 0);
    MFMA8(a1, b1);
  }
  READ_FRAGS(a1, b1, nk - 1, 1);
  MFMA8(a0, b0);
  MFMA8(a1, b1);
#undef ISSUE
#undef READ_FRAGS
#undef MFMA8
}

// Fragment LDS offsets of a wavefront (wm, wn): token rows wm*128 + 32i +
// lane%32; weight rows from the two column tiles brow0, brow1.
__device__ __forceinline__ void frag_offsets(int wm, int brow0, int brow1, int lane,
                                             int (&aoff)[4], int (&asw)[4], int (&boff)[2],
                                             int (&bsw)[2]) {
  const int fr = lane & 31;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int R = wm * 128 + i * 32 + fr;
    aoff[i] = R * 64;
    asw[i] = swz(R);
  }
  boff[0] = STAGE_A + (brow0 + fr) * 64;
  bsw[0] = swz(brow0 + fr);
  boff[1] = STAGE_A + (brow1 + fr) * 64;
  bsw[1] = swz(brow1 + fr);
}

__device__ __forceinline__ void zero_acc(f32x16 (&acc)[4][2]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.0f;
}

// Epilogue modes of the row-grouped kernel.
enum { EPI_SWIGLU = 0, EPI_PLAIN = 1, EPI_AB = 2, EPI_SWIGLU_AB = 3 };

// Row-grouped kernel (rows of each expert against that expert's weights).
//   EPI_SWIGLU: B-tile = 64 W1 rows + the 64 matching W3 rows; stores
//               h = silu(A) * B (bf16, row length f).
//   EPI_PLAIN : B-tile = 128 weight rows; stores the product (bf16).
//   EPI_AB    : as EPI_SWIGLU but stores A and B themselves (bf16, row
//               length 2f: A at column n, B at column f + n).
// GATHER: token row r of the A operand is X[row_map[r]] (the permute is
// recomputed instead of read).
template <int EPI, bool GATHER>
__global__ __launch_bounds__(256, 2) void gemm_bf16_big(
    const bf16_t* __restrict__ A, const int32_t* __restrict__ row_map, int T,
    const bf16_t* __restrict__ B, bf16_t* __restrict__ C, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ tile_start, int E, int N, int K, int f, int Ncols, int n_tiles,
    int grid_total) {
  constexpr bool PAIRED = EPI != EPI_PLAIN;  // B-tile holds W1/W3 halves
  __shared__ __attribute__((aligned(1024))) char lds[DMA_LDS];
  const int b = blockIdx.x;
  const int Lt = xcd_tile(tile_start, E, n_tiles, grid_total, b);
  int e, row0, rows, nt;
  if (!find_tile_grouped(tile_start, offsets, E, GBM, N, n_tiles, Lt, e, row0, rows, nt)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int n0 = nt * (PAIRED ? 64 : 128);
  const size_t Brows_e = PAIRED ? (size_t)2 * f : (size_t)Ncols;
  const bf16_t* Be = B + (size_t)e * Brows_e * K;

  // DMA sources: wavefront wv fills token rows wv*64.. (A_INS instructions
  // of 16 rows x 4 chunks) and weight rows wv*32.. (B_INS); lane -> (row +
  // lane/4, slot lane%4)
  const bf16_t* asrc[A_INS];
  const bf16_t* bsrc[B_INS];
#pragma unroll
  for (int i = 0; i < A_INS; ++i) {
    const int R = wv * (GBM / 4) + i * 16 + (lane >> 2);
    const int c = (lane & 3) ^ swz(R);
    const int r = row0 + min(R, rows - 1);
    const size_t arow = GATHER ? (size_t)min(max(row_map[r], 0), T - 1) : (size_t)r;
    asrc[i] = A + arow * K + c * 8;
  }
#pragma unroll
  for (int i = 0; i < B_INS; ++i) {
    const int R = wv * (GBN / 4) + i * 16 + (lane >> 2);
    const int c = (lane & 3) ^ swz(R);
    const int wrow = PAIRED ? (R < 64 ? n0 + R : f + n0 + (R - 64)) : n0 + R;
    bsrc[i] = Be + (size_t)wrow * K + c * 8;
  }
  int aoff[4], asw[4], boff[2], bsw[2];
  frag_offsets(wm, PAIRED ? wn * 32 : wn * 64, PAIRED ? 64 + wn * 32 : wn * 64 + 32, lane, aoff,
               asw, boff, bsw);
  f32x16 acc[4][2];
  zero_acc(acc);
  mma_pipeline<A_INS, B_INS>(lds, asrc, bsrc, K / GBK, wv, lane, aoff, asw, boff, bsw, acc);
  WAIT_VM_LGKM0(0);
  stage_barrier();

  // epilogue through LDS: lane owns token row (i*32 + lane%32) and columns
  // 8*(q/4) + 4*(lane/32) + (q%4) of each 32-wide column tile
  constexpr int CS = EPI == EPI_SWIGLU ? 64 : 128;
  constexpr int CLD = CS + 8;
  bf16_t* Cs = (bf16_t*)lds;
  const int fr = lane & 31, cbase = (lane >> 5) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rl = wm * 128 + i * 32 + fr;
#pragma unroll
    for (int j = 0; j < (EPI == EPI_SWIGLU ? 1 : 2); ++j) {
      // EPI_AB keeps the A half in columns 0..63 and the B half in 64..127
      const int col0 = EPI == EPI_SWIGLU ? wn * 32 : (EPI == EPI_AB ? j * 64 + wn * 32 : wn * 64 + j * 32);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        bf16x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float x = acc[i][j][g * 4 + q];
          if (EPI == EPI_SWIGLU) {
            const float y = acc[i][1][g * 4 + q];
            v[q] = (bf16_t)(silu(x) * y);
          } else {
            v[q] = (bf16_t)x;
          }
        }
        *(bf16x4*)(Cs + rl * CLD + col0 + g * 8 + cbase) = v;
      }
    }
  }
  __syncthreads();
  constexpr int CPR = CS / 8;  // 16-byte chunks per row
  for (int c = tid; c < GBM * CPR; c += 256) {
    const int rr = c / CPR, cc = (c - rr * CPR) * 8;
    if (rr >= rows) continue;
    size_t col;
    if (EPI == EPI_AB) col = cc < 64 ? (size_t)n0 + cc : (size_t)f + n0 + (cc - 64);
    else col = (size_t)nt * CS + cc;
    *(u32x4*)(C + (size_t)(row0 + rr) * Ncols + col) = *(const u32x4*)(Cs + rr * CLD + cc);
  }
}

// Explicit instantiations: clang's host pass does not emit the launch stubs
// of these kernel templates when they are only instantiated implicitly.
#define MOE_INST_BIG(EPI, GATHER)                                                          \
  template __global__ void gemm_bf16_big<EPI, GATHER>(                                     \
      const bf16_t* __restrict__, const int32_t* __restrict__, int, const bf16_t* __restrict__, \
      bf16_t* __restrict__, const int32_t* __restrict__, const int32_t* __restrict__, int, int, \
      int, int, int, int, int);
MOE_INST_BIG(EPI_SWIGLU, false)
MOE_INST_BIG(EPI_PLAIN, false)
MOE_INST_BIG(EPI_AB, true)
#undef MOE_INST_BIG

// ------------------------------------------------- BF16, 256 x 256 tiles
// Forward expert GEMMs: block tile 256 tokens x 256 weight rows, K = 64 per
// stage (128-byte LDS rows, one full cache line per row and stage), two
// stages of 64 KB, one block per CU with 8 wavefronts (2 rows x 4 columns,
// each 128 x 64 as 4 x 2 tiles of v_mfma_f32_32x32x16_bf16), so two
// wavefronts per SIMD as in the 256 x 128 kernel but half the L2 bytes per
// flop and one barrier per 32 MFMAs.  Chunk swizzle over the eight 16-byte
// chunks of a row: physical = logical ^ ((row >> 1) & 7).  A 128-byte row is
// half of the 64 four-byte LDS banks and a 128-bit fragment read serves 16
// lanes (16 consecutive rows, one chunk each) per cycle, so rows r and r + 8
// must differ in their chunk too; with ^ (row & 7) they met in the same
// banks, a two-way conflict on every read.  SwiGLU: weight rows
// 0..127 are W1 rows n0.., 128..255 the matching W3 rows; wavefront wn owns
// outputs wn*32 .. wn*32+31 (gate tile and up tile).
constexpr int XBN = 256, XBK = 64;
constexpr int XSTAGE_A = GBM * 128, XSTAGE_B = XBN * 128;
constexpr int XSTAGE = XSTAGE_A + XSTAGE_B;
constexpr int XEPI = GBM * (256 + 8) * 2;
constexpr int XLDS = 2 * XSTAGE > XEPI ? 2 * XSTAGE : XEPI;
constexpr int XW = 8;  // wavefronts per block: 2 (rows) x 4 (columns), each 128 x 64
constexpr int XA_INS = GBM * 128 / 1024 / XW, XB_INS = XBN * 128 / 1024 / XW;

// EPI_AB (backward): the SwiGLU tiles, storing A and B themselves (row
// length 2f: A at column n, B at column f + n).  GATHER: token row r of
// the A operand is X[row_map[r]] (the permute recomputed, not read).
// Epilogue of the 256 x 256 tile: the wavefront's 128 x 64 accumulators
// (4 x 2 tiles of 32 x 32) staged through LDS and written as rows of 16-byte
// chunks.  WS_H: h = silu(A) * B of the paired tile (128 columns at
// nt * 128); WS_AB: A in columns 0..127 of the staged tile, B in 128..255,
// stored at n0 + c and f + n0 + c; WS_PLAIN: 256 columns at nt * 256.
enum { WS_H = 0, WS_AB = 1, WS_PLAIN = 2 };
template <int MODE>
__device__ __forceinline__ void wide_store(const f32x16 (&acc)[4][2], char* lds,
                                           bf16_t* __restrict__ C, int Ncols, int rows,
                                           int row0, int n0, int nt, int f) {
  constexpr int CS = MODE == WS_H ? 128 : 256;
  constexpr int CLD = CS + 8;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 2, wn = wv & 3, fr = lane & 31, fh = lane >> 5;
  bf16_t* Cs = (bf16_t*)lds;
  const int cbase = fh * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rl = wm * 128 + i * 32 + fr;
#pragma unroll
    for (int j = 0; j < (MODE == WS_H ? 1 : 2); ++j) {
      const int col0 =
          MODE == WS_H ? wn * 32 : (MODE == WS_AB ? j * 128 + wn * 32 : wn * 64 + j * 32);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        bf16x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float x = acc[i][j][g * 4 + q];
          if (MODE == WS_H) v[q] = (bf16_t)(silu(x) * acc[i][1][g * 4 + q]);
          else v[q] = (bf16_t)x;
        }
        *(bf16x4*)(Cs + rl * CLD + col0 + g * 8 + cbase) = v;
      }
    }
  }
  __syncthreads();
  constexpr int CPR = CS / 8;
  for (int c = tid; c < GBM * CPR; c += 64 * XW) {
    const int rr = c / CPR, cc = (c - rr * CPR) * 8;
    if (rr >= rows) continue;
    size_t col;
    if (MODE == WS_AB) col = cc < 128 ? (size_t)n0 + cc : (size_t)f + n0 + (cc - 128);
    else col = (size_t)nt * CS + cc;
    *(u32x4*)(C + (size_t)(row0 + rr) * Ncols + col) = *(const u32x4*)(Cs + rr * CLD + cc);
  }
}

template <int EPI, bool GATHER>
__global__ __launch_bounds__(64 * XW, 1) void gemm_bf16_wide(
    const bf16_t* __restrict__ A, const int32_t* __restrict__ row_map, int T,
    const bf16_t* __restrict__ B, bf16_t* __restrict__ C, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ tile_start, int E, int N, int K, int f, int Ncols, int n_tiles,
    int grid_total, bf16_t* __restrict__ C2) {
  typedef __attribute__((address_space(3))) void lds_void;
  constexpr bool PAIRED = EPI != EPI_PLAIN;
  __shared__ __attribute__((aligned(1024))) char lds[XLDS];
  const int b = blockIdx.x;
  const int Lt = xcd_tile(tile_start, E, n_tiles, grid_total, b);
  int e, row0, rows, nt;
  if (!find_tile_grouped(tile_start, offsets, E, GBM, N, n_tiles, Lt, e, row0, rows, nt)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 2, wn = wv & 3;
  const int n0 = nt * (PAIRED ? 128 : 256);
  const size_t Brows_e = PAIRED ? (size_t)2 * f : (size_t)Ncols;
  const bf16_t* Be = B + (size_t)e * Brows_e * K;
  const bf16_t* asrc[XA_INS];
  const bf16_t* bsrc[XB_INS];
#pragma unroll
  for (int i = 0; i < XA_INS; ++i) {
    const int R = wv * (GBM / XW) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    const int r = row0 + min(R, rows - 1);
    const size_t arow = GATHER ? (size_t)min(max(row_map[r], 0), T - 1) : (size_t)r;
    asrc[i] = A + arow * K + c * 8;
  }
#pragma unroll
  for (int i = 0; i < XB_INS; ++i) {
    const int R = wv * (XBN / XW) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    const int wrow = PAIRED ? (R < 128 ? n0 + R : f + n0 + (R - 128)) : n0 + R;
    bsrc[i] = Be + (size_t)wrow * K + c * 8;
  }
  const int fr = lane & 31, fh = lane >> 5;
  int aoff[4], asw[4], boff[2], bsw[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int R = wm * 128 + i * 32 + fr;
    aoff[i] = R * 128;
    asw[i] = (R >> 1) & 7;
  }
  // SwiGLU: wavefront wn owns 32 outputs: gate rows wn*32.., up rows 128+wn*32..
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int R = (PAIRED ? (j == 0 ? wn * 32 : 128 + wn * 32) : wn * 64 + j * 32) + fr;
    boff[j] = XSTAGE_A + R * 128;
    bsw[j] = (R >> 1) & 7;
  }
  f32x16 acc[4][2];
  zero_acc(acc);
  const int nk = K / XBK;
#define X_ISSUE(kstep)                                                                         \
  {                                                                                            \
    char* st_ = lds + ((kstep) & 1) * XSTAGE;                                                  \
    const int k0_ = (kstep) * XBK;                                                             \
    _Pragma("unroll") for (int i = 0; i < XA_INS; ++i) __builtin_amdgcn_global_load_lds(       \
        asrc[i] + k0_, (lds_void*)(st_ + (wv * (GBM / XW) + i * 8) * 128), 16, 0, 0);          \
    _Pragma("unroll") for (int i = 0; i < XB_INS; ++i) __builtin_amdgcn_global_load_lds(       \
        bsrc[i] + k0_, (lds_void*)(st_ + XSTAGE_A + (wv * (XBN / XW) + i * 8) * 128), 16, 0,   \
        0);                                                                                    \
  }
#define X_READ(AF, BF, stp, ks)                                                          \
  {                                                                                      \
    const char* st_ = lds + ((stp) & 1) * XSTAGE;                                        \
    const int c_ = (ks) * 2 + fh;                                                        \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) AF[i] =                                \
        *(const bf16x8*)(st_ + aoff[i] + ((c_ ^ asw[i]) << 4));                          \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) BF[j] =                                \
        *(const bf16x8*)(st_ + boff[j] + ((c_ ^ bsw[j]) << 4));                          \
  }
#define X_MFMA(AF, BF)                                                                   \
  _Pragma("unroll") for (int i = 0; i < 4; ++i) _Pragma("unroll") for (int j = 0; j < 2; \
                                                                       ++j) acc[i][j] =  \
      __builtin_amdgcn_mfma_f32_32x32x16_bf16(BF[j], AF[i], acc[i][j], 0, 0, 0);
  bf16x8 a0[4], b0[2], a1[4], b1[2];
  X_ISSUE(0);
  if (nk > 1) {
    X_ISSUE(1);
    WAIT_VM_LGKM0(XA_INS + XB_INS);
  } else {
    WAIT_VM_LGKM0(0);
  }
  stage_barrier();
  X_READ(a0, b0, 0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    // LLVM's single-wavefront MFMA interleave strategy for the loop body
    // (measured 5-8% faster on both forward products)
    __builtin_amdgcn_iglp_opt(1);
    X_READ(a1, b1, kt, 1);
    X_MFMA(a0, b0);
    X_READ(a0, b0, kt, 2);
    X_MFMA(a1, b1);
    X_READ(a1, b1, kt, 3);
    X_MFMA(a0, b0);
    WAIT_VM_LGKM0(0);
    stage_barrier();
    if (kt + 2 < nk) X_ISSUE(kt + 2);
    if (kt + 1 < nk) X_READ(a0, b0, kt + 1, 0);
    X_MFMA(a1, b1);
  }
#undef X_ISSUE
#undef X_READ
#undef X_MFMA
  WAIT_VM_LGKM0(0);
  stage_barrier();

  // SwiGLU: 128 h columns per tile; EPI_AB: A and B; plain: 256 columns;
  // EPI_SWIGLU_AB: h into C, then A and B into C2 (row length 2f)
  wide_store<(EPI == EPI_SWIGLU || EPI == EPI_SWIGLU_AB) ? WS_H : (EPI == EPI_AB ? WS_AB : WS_PLAIN)>(
      acc, lds, C, Ncols, rows, row0, n0, nt, f);
  if (EPI == EPI_SWIGLU_AB) {
    __syncthreads();  // every thread is done reading the h tile
    wide_store<WS_AB>(acc, lds, C2, 2 * f, rows, row0, n0, nt, f);
  }
}

// ------------------------------------- BF16 MFMA, 256x256, K-major B
// The plain product C[r] = A[r] B_e with B_e stored K-major, [K, Ncols] row
// by row (a weight matrix as it is stored, e.g. W2_e [d, f] for U = dY W2_e),
// so no transposed copy of B is made.  A, the tiles, the wavefront layout,
// the two-stage ring and the epilogue are those of gemm_bf16_wide.  A stage
// holds 64 K-rows of 256 B-columns (512 bytes each); the 16-byte chunks of
// K-row k are stored at chunk ^ 4 (k & 3), so the transpose reads below hit
// distinct LDS banks within each half-wavefront.  A B fragment (32 columns
// x 16 K) is two ds_read_b64_tr_b16: within a group of 16 lanes, lane i
// receives element i % 4 of the 8-byte pieces the group's lanes 4q + i / 4
// (q = 0..3) point at; lane p of the group points at K-row kb + p / 4 and
// columns c + 4 (p % 4) .. + 3, so lane i holds four consecutive K of
// column c + i.
typedef short v4s_t __attribute__((ext_vector_type(4)));
typedef short v8s_t __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) v4s_t lds_v4s_t;

__device__ __forceinline__ int bkm_off(int k, int n) {
  return k * 512 + ((((n >> 3) ^ (4 * (k & 3))) & 31) << 4) + ((n & 7) << 1);
}

__global__ __launch_bounds__(64 * XW, 1) void gemm_bf16_wide_bkm(
    const bf16_t* __restrict__ A, const bf16_t* __restrict__ B, bf16_t* __restrict__ C,
    const int32_t* __restrict__ offsets, const int32_t* __restrict__ tile_start, int E, int N,
    int K, int Ncols, int n_tiles, int grid_total) {
  typedef __attribute__((address_space(3))) void lds_void;
  __shared__ __attribute__((aligned(1024))) char lds[XLDS];
  const int b = blockIdx.x;
  const int Lt = xcd_tile(tile_start, E, n_tiles, grid_total, b);
  int e, row0, rows, nt;
  if (!find_tile_grouped(tile_start, offsets, E, GBM, N, n_tiles, Lt, e, row0, rows, nt)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 2, wn = wv & 3;
  const int n0 = nt * 256;
  const bf16_t* Be = B + (size_t)e * K * Ncols;
  const bf16_t* asrc[XA_INS];
  const bf16_t* bsrc[XB_INS];
#pragma unroll
  for (int i = 0; i < XA_INS; ++i) {
    const int R = wv * (GBM / XW) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    asrc[i] = A + (size_t)(row0 + min(R, rows - 1)) * K + c * 8;
  }
  // B: instruction i of wavefront wv fills K-rows 8 wv + 2 i (lanes 0..31)
  // and 8 wv + 2 i + 1 (lanes 32..63), lane chunk c at physical chunk c
#pragma unroll
  for (int i = 0; i < XB_INS; ++i) {
    const int kr = wv * 8 + i * 2 + (lane >> 5);
    const int c = (lane & 31) ^ (4 * (kr & 3));
    bsrc[i] = Be + (size_t)kr * Ncols + n0 + c * 8;
  }
  const int fr = lane & 31, fh = lane >> 5;
  int aoff[4], asw[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int R = wm * 128 + i * 32 + fr;
    aoff[i] = R * 128;
    asw[i] = (R >> 1) & 7;
  }
  // transpose-read offsets of the two B fragments (kk = 0; +4 K-rows for
  // the second read), relative to the stage and the 16-K step
  const int g = lane >> 4, p = lane & 15;
  int boff[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int h = 0; h < 2; ++h)
      boff[j][h] = bkm_off(8 * (g >> 1) + 4 * h + (p >> 2), wn * 64 + j * 32 + 16 * (g & 1) + 4 * (p & 3));
  f32x16 acc[4][2];
  zero_acc(acc);
  const int nk = K / XBK;
#define K_ISSUE(kstep)                                                                         \
  {                                                                                            \
    char* st_ = lds + ((kstep) & 1) * XSTAGE;                                                  \
    const int k0_ = (kstep) * XBK;                                                             \
    _Pragma("unroll") for (int i = 0; i < XA_INS; ++i) __builtin_amdgcn_global_load_lds(       \
        asrc[i] + k0_, (lds_void*)(st_ + (wv * (GBM / XW) + i * 8) * 128), 16, 0, 0);          \
    _Pragma("unroll") for (int i = 0; i < XB_INS; ++i) __builtin_amdgcn_global_load_lds(       \
        bsrc[i] + (size_t)k0_ * Ncols, (lds_void*)(st_ + XSTAGE_A + (wv * 8 + i * 2) * 512),   \
        16, 0, 0);                                                                             \
  }
  // the K-row of a B fragment read moves by 16 per K step: 16 * 512 bytes,
  // with (k & 3) unchanged, so the swizzle of the offsets above still holds
#define K_READ(AF, BF, stp, ks)                                                              \
  {                                                                                          \
    const char* st_ = lds + ((stp) & 1) * XSTAGE;                                            \
    const int c_ = (ks) * 2 + fh;                                                            \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) AF[i] =                                    \
        *(const bf16x8*)(st_ + aoff[i] + ((c_ ^ asw[i]) << 4));                              \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) {                                          \
      const char* bb_ = st_ + XSTAGE_A + (ks) * 16 * 512;                                \
      const v4s_t lo_ = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s_t*)(bb_ + boff[j][0])); \
      const v4s_t hi_ = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s_t*)(bb_ + boff[j][1])); \
      BF[j] = __builtin_bit_cast(bf16x8, (v8s_t){lo_[0], lo_[1], lo_[2], lo_[3], hi_[0], hi_[1], hi_[2], hi_[3]}); \
    }                                                                                        \
  }
#define K_MFMA(AF, BF)                                                                   \
  _Pragma("unroll") for (int i = 0; i < 4; ++i) _Pragma("unroll") for (int j = 0; j < 2; \
                                                                       ++j) acc[i][j] =  \
      __builtin_amdgcn_mfma_f32_32x32x16_bf16(BF[j], AF[i], acc[i][j], 0, 0, 0);
  bf16x8 a0[4], b0[2], a1[4], b1[2];
  K_ISSUE(0);
  if (nk > 1) {
    K_ISSUE(1);
    WAIT_VM_LGKM0(XA_INS + XB_INS);
  } else {
    WAIT_VM_LGKM0(0);
  }
  stage_barrier();
  K_READ(a0, b0, 0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_iglp_opt(1);
    K_READ(a1, b1, kt, 1);
    K_MFMA(a0, b0);
    K_READ(a0, b0, kt, 2);
    K_MFMA(a1, b1);
    K_READ(a1, b1, kt, 3);
    K_MFMA(a0, b0);
    WAIT_VM_LGKM0(0);
    stage_barrier();
    if (kt + 2 < nk) K_ISSUE(kt + 2);
    if (kt + 1 < nk) K_READ(a0, b0, kt + 1, 0);
    K_MFMA(a1, b1);
  }
#undef K_ISSUE
#undef K_READ
#undef K_MFMA
  WAIT_VM_LGKM0(0);
  stage_barrier();
  wide_store<WS_PLAIN>(acc, lds, C, Ncols, rows, row0, 0, nt, 0);
}

#define MOE_INST_WIDE(EPI, GATHER)                                                          \
  template __global__ void gemm_bf16_wide<EPI, GATHER>(                                     \
      const bf16_t* __restrict__, const int32_t* __restrict__, int, const bf16_t* __restrict__, \
      bf16_t* __restrict__, const int32_t* __restrict__, const int32_t* __restrict__, int, int, \
      int, int, int, int, int, bf16_t* __restrict__);
MOE_INST_WIDE(EPI_SWIGLU, false)
MOE_INST_WIDE(EPI_SWIGLU, true)
MOE_INST_WIDE(EPI_SWIGLU_AB, true)
MOE_INST_WIDE(EPI_PLAIN, false)
MOE_INST_WIDE(EPI_AB, true)
#undef MOE_INST_WIDE

// ------------------------------------------------------------------ FP8
// Per-block FP8 e4m3 quantisation (block amax, inv = 448 / amax, codes of
// x * inv, scale = amax / 448; an all-zero block has scale 1 and codes 0).

// 1 x 128 blocks: one wavefront per row, 16 lanes of 8 values per block.
template <typename TA>
__global__ __launch_bounds__(256) void fp8_quant_rows(const TA* __restrict__ X, int R, int C,
                                                      fp8_t* __restrict__ Q,
                                                      float* __restrict__ S) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= R) return;
  const int nblk = C / 128;
  for (int c0 = 0; c0 < C; c0 += 512) {
    const int col = c0 + lane * 8;
    const bool act = col < C;
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = act ? ActIO<TA>::ld(X + (size_t)r * C + col, i) : 0.0f;
    float am = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) am = fmaxf(am, fabsf(v[i]));
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) am = fmaxf(am, __shfl_xor(am, o, 64));
    const bool nz = am > 0.0f;
    const float inv = nz ? 448.0f / am : 1.0f;
    u32x2 q;
    q[0] = q[1] = 0u;
    if (nz) {
      q[0] = fp8_encode4(v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv);
      q[1] = fp8_encode4(v[4] * inv, v[5] * inv, v[6] * inv, v[7] * inv);
    }
    if (act) {
      *(u32x2*)(Q + (size_t)r * C + col) = q;
      if ((lane & 15) == 0) S[(size_t)r * nblk + col / 128] = nz ? am / 448.0f : 1.0f;
    }
  }
}

// 128 x 128 blocks (ragged last row block): one 256-thread block per tile.
template <typename TA>
__global__ __launch_bounds__(256) void fp8_quant_tiles(const TA* __restrict__ X, int R, int C,
                                                       fp8_t* __restrict__ Q,
                                                       float* __restrict__ S) {
  __shared__ float red[256];
  const int tid = threadIdx.x;
  const int cb = blockIdx.x, rb = blockIdx.y;
  const int r0 = rb * 128, nr = min(128, R - r0);
  const int col = cb * 128 + (tid & 15) * 8;
  float am = 0.0f;
  for (int rr = tid >> 4; rr < nr; rr += 16)
#pragma unroll
    for (int i = 0; i < 8; ++i)
      am = fmaxf(am, fabsf(ActIO<TA>::ld(X + (size_t)(r0 + rr) * C + col, i)));
  red[tid] = am;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) red[tid] = fmaxf(red[tid], red[tid + h]);
    __syncthreads();
  }
  am = red[0];
  const bool nz = am > 0.0f;
  const float inv = nz ? 448.0f / am : 1.0f;
  for (int rr = tid >> 4; rr < nr; rr += 16) {
    u32x2 q;
    q[0] = q[1] = 0u;
    if (nz) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        q[i >> 2] |= fp8_encode(ActIO<TA>::ld(X + (size_t)(r0 + rr) * C + col, i) * inv)
                     << (8 * (i & 3));
    }
    *(u32x2*)(Q + (size_t)(r0 + rr) * C + col) = q;
  }
  if (tid == 0) S[(size_t)rb * (C / 128) + cb] = nz ? am / 448.0f : 1.0f;
}

typedef int i32x8 __attribute__((ext_vector_type(8)));

// FP8 grouped GEMM 2 when d % 256 != 0, with per-block scales: A codes
// [N,K] (h) with scales [N, K/128] (1 x 128 blocks), B codes [E, Ncols, K]
// with scales
// [E, Ncols/128, K/128] (128 x 128 blocks).  Tiles and tile order as
// gemm_bf16_big (256 tokens x 128 weight rows, 4 wavefronts of 128 x 64);
// one stage is one 128-wide K block: 128-byte LDS rows (a full cache line
// per row) with the chunk swizzle physical = logical ^ ((row >> 1) & 7) of
// the 256 x 256 kernel (conflict-free 128-bit fragment reads), three
// stages of 48 KB, one block per CU.  Per stage and 32x32 tile, two
// v_mfma_f32_32x32x64_f8f6f4 accumulate the block on its own, which is then
// promoted into the FP32 result: acc += partial * (sa * sb).  A lane holds
// one token row of each tile, so sa is one value per row tile and sb one
// value per column tile (wavefront-uniform).
constexpr int F8_STAGE_A = GBM * 128, F8_STAGE_B = GBN * 128;
constexpr int F8_STAGE = F8_STAGE_A + F8_STAGE_B;
constexpr int F8_NSTAGE = 3;
constexpr int F8_LDS = F8_NSTAGE * F8_STAGE > EPI_BYTES ? F8_NSTAGE * F8_STAGE : EPI_BYTES;
constexpr int F8_A_INS = GBM * 128 / 1024 / 4, F8_B_INS = GBN * 128 / 1024 / 4;

__global__ __launch_bounds__(256, 1) void gemm_fp8_big(
    const fp8_t* __restrict__ A, const float* __restrict__ As, const fp8_t* __restrict__ B,
    const float* __restrict__ Bs, bf16_t* __restrict__ C, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ tile_start, int E, int N, int K, int Ncols, int n_tiles,
    int grid_total) {
  typedef __attribute__((address_space(3))) void lds_void;
  __shared__ __attribute__((aligned(1024))) char lds[F8_LDS];
  const int b = blockIdx.x;
  const int Lt = xcd_tile(tile_start, E, n_tiles, grid_total, b);
  int e, row0, rows, nt;
  if (!find_tile_grouped(tile_start, offsets, E, GBM, N, n_tiles, Lt, e, row0, rows, nt)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = __builtin_amdgcn_readfirstlane(wv & 1);
  const int n0 = nt * 128;
  const int Brows_e = Ncols;
  const int nkb = K / 128;
  const fp8_t* Be = B + (size_t)e * Brows_e * K;
  // DMA: one instruction = 8 rows x 128 bytes; lane -> (row + lane/8,
  // physical chunk lane%8)
  const fp8_t* asrc[F8_A_INS];
  const fp8_t* bsrc[F8_B_INS];
#pragma unroll
  for (int i = 0; i < F8_A_INS; ++i) {
    const int R = wv * (GBM / 4) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    const size_t arow = (size_t)(row0 + min(R, rows - 1));
    asrc[i] = A + arow * K + c * 16;
  }
#pragma unroll
  for (int i = 0; i < F8_B_INS; ++i) {
    const int R = wv * (GBN / 4) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    const int wrow = n0 + R;
    bsrc[i] = Be + (size_t)wrow * K + c * 16;
  }
  const int fr = lane & 31, fh = lane >> 5;
  int aoff[4], asw[4], boff[2], bsw[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int R = wm * 128 + i * 32 + fr;
    aoff[i] = R * 128;
    asw[i] = (R >> 1) & 7;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int R = wn * 64 + j * 32 + fr;
    boff[j] = F8_STAGE_A + R * 128;
    bsw[j] = (R >> 1) & 7;
  }
  // scale rows: token rows of the lane in each row tile, weight row blocks
  // of the wavefront's two column tiles
  const float* sa_row[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sa_row[i] = As + (size_t)(row0 + min(wm * 128 + i * 32 + fr, rows - 1)) * nkb;
  }
  const int wr0 = n0 + wn * 64, wr1 = n0 + wn * 64 + 32;
  const float* sb_row0 = Bs + ((size_t)e * (Brows_e / 128) + wr0 / 128) * nkb;
  const float* sb_row1 = Bs + ((size_t)e * (Brows_e / 128) + wr1 / 128) * nkb;

  f32x16 acc[4][2], part[4][2];
  zero_acc(acc);
  zero_acc(part);
  const int nk = nkb;
  constexpr int VMS = F8_A_INS + F8_B_INS;
#define F8_ISSUE(kstep)                                                                        \
  {                                                                                            \
    char* st_ = lds + ((kstep) % F8_NSTAGE) * F8_STAGE;                                        \
    const int k0_ = (kstep) * 128;                                                             \
    _Pragma("unroll") for (int i = 0; i < F8_A_INS; ++i) __builtin_amdgcn_global_load_lds(     \
        asrc[i] + k0_, (lds_void*)(st_ + (wv * (GBM / 4) + i * 8) * 128), 16, 0, 0);           \
    _Pragma("unroll") for (int i = 0; i < F8_B_INS; ++i) __builtin_amdgcn_global_load_lds(     \
        bsrc[i] + k0_, (lds_void*)(st_ + F8_STAGE_A + (wv * (GBN / 4) + i * 8) * 128), 16, 0,  \
        0);                                                                                    \
  }
  // K half h of a stage: chunks 4h + fh and 4h + 2 + fh of each row
#define F8_READ(AF, BF, stp, h)                                                               \
  {                                                                                           \
    const char* st_ = lds + ((stp) % F8_NSTAGE) * F8_STAGE;                                   \
    const int c0_ = 4 * (h) + fh, c1_ = 4 * (h) + 2 + fh;                                     \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                           \
      const u32x4 lo_ = *(const u32x4*)(st_ + aoff[i] + ((c0_ ^ asw[i]) << 4));               \
      const u32x4 hi_ = *(const u32x4*)(st_ + aoff[i] + ((c1_ ^ asw[i]) << 4));               \
      AF[i] = (i32x8){(int)lo_[0], (int)lo_[1], (int)lo_[2], (int)lo_[3],                     \
                      (int)hi_[0], (int)hi_[1], (int)hi_[2], (int)hi_[3]};                    \
    }                                                                                         \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) {                                           \
      const u32x4 lo_ = *(const u32x4*)(st_ + boff[j] + ((c0_ ^ bsw[j]) << 4));               \
      const u32x4 hi_ = *(const u32x4*)(st_ + boff[j] + ((c1_ ^ bsw[j]) << 4));               \
      BF[j] = (i32x8){(int)lo_[0], (int)lo_[1], (int)lo_[2], (int)lo_[3],                     \
                      (int)hi_[0], (int)hi_[1], (int)hi_[2], (int)hi_[3]};                    \
    }                                                                                         \
  }
#define F8_MFMA(AF, BF)                                                                       \
  _Pragma("unroll") for (int i = 0; i < 4; ++i) _Pragma("unroll") for (int j = 0; j < 2; ++j) \
      part[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(BF[j], AF[i], part[i][j], \
                                                                    0, 0, 0, 0, 0, 0);
#define F8_WAITN(n_)                         \
  switch (n_) {                              \
    case 0: WAIT_VM_LGKM0(0); break;         \
    case 1: WAIT_VM_LGKM0(VMS); break;       \
    default: WAIT_VM_LGKM0(2 * VMS); break;  \
  }
  i32x8 a0[4], b0[2], a1[4], b1[2];
  float sa[4], sb[2], san[4], sbn[2];
  const int pre = nk < F8_NSTAGE ? nk : F8_NSTAGE;
  for (int s_ = 0; s_ < pre; ++s_) F8_ISSUE(s_);
#pragma unroll
  for (int i = 0; i < 4; ++i) san[i] = sa_row[i][0];
  sbn[0] = sb_row0[0];
  sbn[1] = sb_row1[0];
  F8_WAITN(pre - 1);
  stage_barrier();
  F8_READ(a0, b0, 0, 0);
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) sa[i] = san[i];
    sb[0] = sbn[0];
    sb[1] = sbn[1];
    F8_READ(a1, b1, kt, 1);
    F8_MFMA(a0, b0);
    if (kt + 1 < nk) {
      // stage kt+1 landed; every wavefront is done reading stage kt
      const int last = nk - 1 < kt + F8_NSTAGE - 1 ? nk - 1 : kt + F8_NSTAGE - 1;
      F8_WAITN(last - (kt + 1));
      stage_barrier();
      // next block's scales go out before the next DMA issue, so the
      // following vmcnt waits cover them without waiting for that issue
#pragma unroll
      for (int i = 0; i < 4; ++i) san[i] = sa_row[i][kt + 1];
      sbn[0] = sb_row0[kt + 1];
      sbn[1] = sb_row1[kt + 1];
      if (kt + F8_NSTAGE < nk) F8_ISSUE(kt + F8_NSTAGE);
      F8_READ(a0, b0, kt + 1, 0);
    }
    F8_MFMA(a1, b1);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float sc = sa[i] * sb[j];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          acc[i][j][q] = fmaf(part[i][j][q], sc, acc[i][j][q]);
          part[i][j][q] = 0.0f;
        }
      }
  }
#undef F8_ISSUE
#undef F8_READ
#undef F8_MFMA
#undef F8_WAITN
  WAIT_VM_LGKM0(0);
  stage_barrier();

  constexpr int CS = 128;
  constexpr int CLD = CS + 8;
  bf16_t* Cs = (bf16_t*)lds;
  const int cbase = (lane >> 5) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rl = wm * 128 + i * 32 + fr;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col0 = wn * 64 + j * 32;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        bf16x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (bf16_t)acc[i][j][g * 4 + q];
        *(bf16x4*)(Cs + rl * CLD + col0 + g * 8 + cbase) = v;
      }
    }
  }
  __syncthreads();
  constexpr int CPR = CS / 8;
  for (int c = tid; c < GBM * CPR; c += 256) {
    const int rr = c / CPR, cc = (c - rr * CPR) * 8;
    if (rr >= rows) continue;
    *(u32x4*)(C + (size_t)(row0 + rr) * Ncols + (size_t)nt * CS + cc) =
        *(const u32x4*)(Cs + rr * CLD + cc);
  }
}


// FP8 expert products on a 128-token x 256-weight-row tile with 8
// wavefronts, two per SIMD, so one wavefront's per-K-block promotion FMAs
// run under the other's MFMAs (one wavefront per SIMD, as in gemm_fp8_big,
// serialises them).  Each wavefront holds 2 x 2 tiles of 32x32 (64 tokens)
// with a block and a running accumulator set (128 + 128 registers).
// Stages, swizzle and per-K-block promotion are those of gemm_fp8_big.
//   GEMM 1 (PLAIN false): weight rows W1 n0..n0+127 and their W3 partners,
//     wavefront (wm, wn) = 64 tokens x h columns wn*32..wn*32+31 (W1 tile
//     j = 0, W3 tile j = 1), so a tile owns whole 1 x 128 blocks of h and
//     writes its codes and scales directly (no BF16 h round trip): h is the
//     BF16 rounding of silu(A) * B, quantised exactly as fp8_quant_rows
//     does (block amax, inverse, codes, scale); a token row's amax meets in
//     LDS from a lane, its partner lane (lane ^ 32) and the other three
//     column-quarter wavefronts.
//   GEMM 2 (PLAIN true): 256 consecutive weight rows (output columns, f is
//     the output width), wavefront = 64 tokens x 64 columns; Y stored in
//     BF16 through LDS.
// GATHER: token row r of the A operand (codes and scales) is row
// row_map[r] of the per-token arrays (the permute fused into the DMA).
constexpr int FQ_BM = 128, FQ_BN = 256;
constexpr int FQ_STAGE_A = FQ_BM * 128, FQ_STAGE_B = FQ_BN * 128;
constexpr int FQ_STAGE = FQ_STAGE_A + FQ_STAGE_B;
constexpr int FQ_W = 8;  // wavefronts: 2 (token halves) x 4 (column quarters)
constexpr int FQ_A_INS = FQ_BM * 128 / 1024 / FQ_W, FQ_B_INS = FQ_BN * 128 / 1024 / FQ_W;
constexpr int FQ_CLD = 144;  // bytes per staged code row (16-byte aligned)
static_assert(FQ_BM * FQ_CLD + 4 * FQ_BM * 4 <= F8_NSTAGE * FQ_STAGE, "epilogue fits the ring");

template <bool GATHER, bool PLAIN>
__global__ __launch_bounds__(512, 1) void gemm_fp8_q(
    const fp8_t* __restrict__ A, const float* __restrict__ As,
    const int32_t* __restrict__ row_map, int T, const fp8_t* __restrict__ B,
    const float* __restrict__ Bs, fp8_t* __restrict__ Hq, float* __restrict__ Hs,
    bf16_t* __restrict__ Y, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ tile_start, int E, int N, int K, int f, int n_tiles,
    int grid_total) {
  typedef __attribute__((address_space(3))) void lds_void;
  __shared__ __attribute__((aligned(1024))) char lds[F8_NSTAGE * FQ_STAGE];
  const int b = blockIdx.x;
  const int Lt = xcd_tile(tile_start, E, n_tiles, grid_total, b);
  int e, row0, rows, nt;
  if (!find_tile_grouped(tile_start, offsets, E, FQ_BM, N, n_tiles, Lt, e, row0, rows, nt))
    return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 2, wn = __builtin_amdgcn_readfirstlane(wv & 3);
  const int n0 = nt * (PLAIN ? 256 : 128);
  const int nkb = K / 128;
  const int Brows_e = PLAIN ? f : 2 * f;  // PLAIN: f is the output width
  const fp8_t* Be = B + (size_t)e * Brows_e * K;
  const fp8_t* asrc[FQ_A_INS];
  const fp8_t* bsrc[FQ_B_INS];
#pragma unroll
  for (int i = 0; i < FQ_A_INS; ++i) {
    const int R = wv * (FQ_BM / FQ_W) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    const int r = row0 + min(R, rows - 1);
    const size_t arow = GATHER ? (size_t)min(max(row_map[r], 0), T - 1) : (size_t)r;
    asrc[i] = A + arow * K + c * 16;
  }
#pragma unroll
  for (int i = 0; i < FQ_B_INS; ++i) {
    const int R = wv * (FQ_BN / FQ_W) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    const int wrow = PLAIN ? n0 + R : (R < 128 ? n0 + R : f + n0 + (R - 128));
    bsrc[i] = Be + (size_t)wrow * K + c * 16;
  }
  const int fr = lane & 31, fh = lane >> 5;
  int aoff[2], asw[2], boff[2], bsw[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int R = wm * 64 + i * 32 + fr;
    aoff[i] = R * 128;
    asw[i] = (R >> 1) & 7;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    // SwiGLU: W1 rows, then their W3 partners; plain: 64 consecutive rows
    const int R = (PLAIN ? wn * 64 + j * 32 : j * 128 + wn * 32) + fr;
    boff[j] = FQ_STAGE_A + R * 128;
    bsw[j] = (R >> 1) & 7;
  }
  const float* sa_row[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int r = row0 + min(wm * 64 + i * 32 + fr, rows - 1);
    const size_t arow = GATHER ? (size_t)min(max(row_map[r], 0), T - 1) : (size_t)r;
    sa_row[i] = As + arow * nkb;
  }
  // weight scale rows: the W1 block and the W3 block of the tile; plain:
  // the block of the wavefront's 64 rows (both of its column tiles)
  const float* sb_row0 =
      Bs + ((size_t)e * (Brows_e / 128) + (PLAIN ? n0 + wn * 64 : n0) / 128) * nkb;
  const float* sb_row1 =
      PLAIN ? sb_row0 : Bs + ((size_t)e * (Brows_e / 128) + (f + n0) / 128) * nkb;

  f32x16 acc[2][2], part[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[i][j][q] = part[i][j][q] = 0.0f;
  const int nk = nkb;
  constexpr int VMS = FQ_A_INS + FQ_B_INS;
#define FQ_ISSUE(kstep)                                                                        \
  {                                                                                            \
    char* st_ = lds + ((kstep) % F8_NSTAGE) * FQ_STAGE;                                        \
    const int k0_ = (kstep) * 128;                                                             \
    _Pragma("unroll") for (int i = 0; i < FQ_A_INS; ++i) __builtin_amdgcn_global_load_lds(     \
        asrc[i] + k0_, (lds_void*)(st_ + (wv * (FQ_BM / FQ_W) + i * 8) * 128), 16, 0, 0);      \
    _Pragma("unroll") for (int i = 0; i < FQ_B_INS; ++i) __builtin_amdgcn_global_load_lds(     \
        bsrc[i] + k0_, (lds_void*)(st_ + FQ_STAGE_A + (wv * (FQ_BN / FQ_W) + i * 8) * 128), 16,\
        0, 0);                                                                                 \
  }
#define FQ_READ(AF, BF, stp, h)                                                               \
  {                                                                                           \
    const char* st_ = lds + ((stp) % F8_NSTAGE) * FQ_STAGE;                                   \
    const int c0_ = 4 * (h) + fh, c1_ = 4 * (h) + 2 + fh;                                     \
    _Pragma("unroll") for (int i = 0; i < 2; ++i) {                                           \
      const u32x4 lo_ = *(const u32x4*)(st_ + aoff[i] + ((c0_ ^ asw[i]) << 4));               \
      const u32x4 hi_ = *(const u32x4*)(st_ + aoff[i] + ((c1_ ^ asw[i]) << 4));               \
      AF[i] = (i32x8){(int)lo_[0], (int)lo_[1], (int)lo_[2], (int)lo_[3],                     \
                      (int)hi_[0], (int)hi_[1], (int)hi_[2], (int)hi_[3]};                    \
    }                                                                                         \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) {                                           \
      const u32x4 lo_ = *(const u32x4*)(st_ + boff[j] + ((c0_ ^ bsw[j]) << 4));               \
      const u32x4 hi_ = *(const u32x4*)(st_ + boff[j] + ((c1_ ^ bsw[j]) << 4));               \
      BF[j] = (i32x8){(int)lo_[0], (int)lo_[1], (int)lo_[2], (int)lo_[3],                     \
                      (int)hi_[0], (int)hi_[1], (int)hi_[2], (int)hi_[3]};                    \
    }                                                                                         \
  }
#define FQ_MFMA(AF, BF)                                                                       \
  _Pragma("unroll") for (int i = 0; i < 2; ++i) _Pragma("unroll") for (int j = 0; j < 2; ++j) \
      part[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(BF[j], AF[i], part[i][j], \
                                                                    0, 0, 0, 0, 0, 0);
#define FQ_WAITN(n_)                         \
  switch (n_) {                              \
    case 0: WAIT_VM_LGKM0(0); break;         \
    case 1: WAIT_VM_LGKM0(VMS); break;       \
    default: WAIT_VM_LGKM0(2 * VMS); break;  \
  }
  i32x8 a0[2], b0[2], a1[2], b1[2];
  float sa[2], sb[2], san[2], sbn[2];
  const int pre = nk < F8_NSTAGE ? nk : F8_NSTAGE;
  for (int s_ = 0; s_ < pre; ++s_) FQ_ISSUE(s_);
#pragma unroll
  for (int i = 0; i < 2; ++i) san[i] = sa_row[i][0];
  sbn[0] = sb_row0[0];
  sbn[1] = sb_row1[0];
  FQ_WAITN(pre - 1);
  stage_barrier();
  FQ_READ(a0, b0, 0, 0);
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int i = 0; i < 2; ++i) sa[i] = san[i];
    sb[0] = sbn[0];
    sb[1] = sbn[1];
    FQ_READ(a1, b1, kt, 1);
    FQ_MFMA(a0, b0);
    if (kt + 1 < nk) {
      const int last = nk - 1 < kt + F8_NSTAGE - 1 ? nk - 1 : kt + F8_NSTAGE - 1;
      FQ_WAITN(last - (kt + 1));
      stage_barrier();
#pragma unroll
      for (int i = 0; i < 2; ++i) san[i] = sa_row[i][kt + 1];
      sbn[0] = sb_row0[kt + 1];
      sbn[1] = sb_row1[kt + 1];
      if (kt + F8_NSTAGE < nk) FQ_ISSUE(kt + F8_NSTAGE);
      FQ_READ(a0, b0, kt + 1, 0);
    }
    FQ_MFMA(a1, b1);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float sc = sa[i] * sb[j];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          acc[i][j][q] = fmaf(part[i][j][q], sc, acc[i][j][q]);
          part[i][j][q] = 0.0f;
        }
      }
  }
#undef FQ_ISSUE
#undef FQ_READ
#undef FQ_MFMA
#undef FQ_WAITN
  WAIT_VM_LGKM0(0);
  stage_barrier();

  if (PLAIN) {
    // Y tile (BF16) through LDS: lane holds token row wm*64 + 32 i + fr,
    // columns wn*64 + 32 j + 8 (q/4) + 4 fh + q%4
    constexpr int YLD = 256 + 8;
    bf16_t* Ys = (bf16_t*)lds;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          bf16x4 v;
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = (bf16_t)acc[i][j][g * 4 + q];
          *(bf16x4*)(Ys + (wm * 64 + i * 32 + fr) * YLD + wn * 64 + j * 32 + g * 8 + fh * 4) = v;
        }
    __syncthreads();
    for (int c = tid; c < FQ_BM * 32; c += 64 * FQ_W) {
      const int rr = c >> 5, cc = (c & 31) * 8;
      if (rr >= rows) continue;
      *(u32x4*)(Y + (size_t)(row0 + rr) * f + n0 + cc) = *(const u32x4*)(Ys + rr * YLD + cc);
    }
    return;
  }

  // h = silu(A) * B rounded to BF16 (lane: token row wm*64 + 32 i + fr,
  // h columns wn*32 + 8 (q/4) + 4 fh + q%4 of the tile), the row's amax
  // over the 128 columns, then the codes through LDS
  uint8_t* Cs = (uint8_t*)lds;
  float* red = (float*)(lds + FQ_BM * FQ_CLD);  // [FQ_W / 2][FQ_BM]
  float hv[2][16];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    float m = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const float v = (float)(bf16_t)(silu(acc[i][0][q]) * acc[i][1][q]);
      hv[i][q] = v;
      m = fmaxf(m, fabsf(v));
    }
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    if (fh == 0) red[wn * FQ_BM + wm * 64 + i * 32 + fr] = m;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int rl = wm * 64 + i * 32 + fr;
    const float a = fmaxf(fmaxf(red[rl], red[FQ_BM + rl]),
                          fmaxf(red[2 * FQ_BM + rl], red[3 * FQ_BM + rl]));
    const bool nz = a > 0.0f;
    const float inv = nz ? 448.0f / a : 1.0f;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      uint32_t w = 0u;
      if (nz)
        w = fp8_encode4(hv[i][g * 4] * inv, hv[i][g * 4 + 1] * inv, hv[i][g * 4 + 2] * inv,
                        hv[i][g * 4 + 3] * inv);
      *(uint32_t*)(Cs + rl * FQ_CLD + wn * 32 + g * 8 + fh * 4) = w;
    }
    if (wn == 0 && fh == 0 && rl < rows)
      Hs[(size_t)(row0 + rl) * (f / 128) + nt] = nz ? a / 448.0f : 1.0f;
  }
  __syncthreads();
  for (int c = tid; c < FQ_BM * 8; c += 64 * FQ_W) {
    const int rr = c >> 3, cc = (c & 7) * 16;
    if (rr >= rows) continue;
    *(u32x4*)(Hq + (size_t)(row0 + rr) * f + n0 + cc) = *(const u32x4*)(Cs + rr * FQ_CLD + cc);
  }
}
template __global__ void gemm_fp8_q<false, false>(
    const fp8_t* __restrict__, const float* __restrict__, const int32_t* __restrict__, int,
    const fp8_t* __restrict__, const float* __restrict__, fp8_t* __restrict__, float* __restrict__,
    bf16_t* __restrict__, const int32_t* __restrict__, const int32_t* __restrict__, int, int, int,
    int, int, int);
template __global__ void gemm_fp8_q<true, false>(
    const fp8_t* __restrict__, const float* __restrict__, const int32_t* __restrict__, int,
    const fp8_t* __restrict__, const float* __restrict__, fp8_t* __restrict__, float* __restrict__,
    bf16_t* __restrict__, const int32_t* __restrict__, const int32_t* __restrict__, int, int, int,
    int, int, int);
template __global__ void gemm_fp8_q<false, true>(
    const fp8_t* __restrict__, const float* __restrict__, const int32_t* __restrict__, int,
    const fp8_t* __restrict__, const float* __restrict__, fp8_t* __restrict__, float* __restrict__,
    bf16_t* __restrict__, const int32_t* __restrict__, const int32_t* __restrict__, int, int, int,
    int, int, int);

// ============================================================ MX formats
// OCP Microscaling blocks: 32 consecutive elements along K share an E8M0
// scale byte (2^(byte - 127)); elements are e4m3 (MX-FP8), e2m3 (MX-FP6)
// or e2m1 (MX-FP4) codes.  Memory layout of a code row of K elements:
//   e4m3  one code per byte                            (K bytes)
//   e2m3  each block's 32 codes packed 6 bits apart (code i at bits 6i of
//         the block's little-endian bit string) in 24 bytes, then 8 zero
//         bytes of padding                             (K bytes)
//   e2m1  two codes per byte, lower index in the low nibble  (K/2 bytes)
// Template parameter FMT is the matrix instruction's format selector
// (0 e4m3, 2 e2m3, 4 e2m1).

template <int FMT> struct MxFmt;
template <> struct MxFmt<0> {
  static constexpr int EB = 4, MB = 3, BIAS = 7, EMAX = 8;
  static constexpr uint32_t MAXCODE = 0x7E;
  static constexpr float MAXV = 448.0f;
};
template <> struct MxFmt<2> {
  static constexpr int EB = 2, MB = 3, BIAS = 1, EMAX = 2;
  static constexpr uint32_t MAXCODE = 0x1F;
  static constexpr float MAXV = 7.5f;
};
template <> struct MxFmt<4> {
  static constexpr int EB = 2, MB = 1, BIAS = 1, EMAX = 2;
  static constexpr uint32_t MAXCODE = 0x7;
  static constexpr float MAXV = 6.0f;
};

// Bytes of a code row of K elements.
__host__ __device__ constexpr size_t mx_row_bytes(int fmt, size_t K) {
  return fmt == 4 ? K / 2 : K;
}

// Shared exponent of a block: floor(log2 amax) - emax, clamped to the E8M0
// range; 0 for an all-zero block.
template <int FMT>
__device__ __forceinline__ int mx_block_exp(float amax) {
  if (!(amax > 0.0f)) return 0;
  const int s = ilogbf(amax) - MxFmt<FMT>::EMAX;
  return s < -127 ? -127 : (s > 127 ? 127 : s);
}

// Code of y (already divided by the block scale): nearest element value,
// ties to the even mantissa, magnitudes above the largest normal saturated;
// the sign is kept (so -0 and negatives rounding to zero are negative zero).
template <int FMT>
__device__ __forceinline__ uint32_t mx_encode(float y) {
  using F = MxFmt<FMT>;
  const uint32_t sign = (__float_as_uint(y) >> 31) << (F::EB + F::MB);
  const float v = fabsf(y);
  uint32_t mag;
  if (v >= F::MAXV) {
    mag = F::MAXCODE;
  } else {
    int e = v > 0.0f ? ilogbf(v) : 1 - F::BIAS;
    if (e < 1 - F::BIAS) e = 1 - F::BIAS;
    const int n = (int)rintf(ldexpf(v, F::MB - e));  // exact scaling, then RNE
    if (n < (1 << F::MB)) {
      mag = (uint32_t)n;  // subnormal (only reachable at the smallest exponent) or zero
    } else if (n == (2 << F::MB)) {
      mag = (uint32_t)((e + 1 + F::BIAS) << F::MB);
    } else {
      mag = (uint32_t)(((e + F::BIAS) << F::MB) | (n - (1 << F::MB)));
    }
  }
  return sign | mag;
}

// Codes of one 32-element block (values already divided by the scale) in
// the memory layout above: 8 words (e4m3, e2m3 with 2 words of padding) or
// 4 words (e2m1).
template <int FMT>
__device__ __forceinline__ void mx_pack_block(const float (&y)[32], uint32_t (&w)[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) w[q] = 0u;
  if (FMT == 0) {
#pragma unroll
    for (int i = 0; i < 32; ++i) w[i >> 2] |= mx_encode<FMT>(y[i]) << (8 * (i & 3));
  } else if (FMT == 4) {
#pragma unroll
    for (int i = 0; i < 32; ++i) w[i >> 3] |= mx_encode<FMT>(y[i]) << (4 * (i & 7));
  } else {
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const uint64_t v = (uint64_t)mx_encode<FMT>(y[i]) << ((6 * i) & 31);
      w[(6 * i) >> 5] |= (uint32_t)v;
      if (((6 * i) & 31) > 26) w[((6 * i) >> 5) + 1] |= (uint32_t)(v >> 32);
    }
  }
}

// Quantise a block of 32 values: writes its codes at dst (32 or 16 bytes,
// 16-byte aligned) and returns the scale byte.
template <int FMT>
__device__ __forceinline__ uint8_t mx_quant_block(float (&x)[32], uint8_t* dst) {
  float amax = 0.0f;
#pragma unroll
  for (int i = 0; i < 32; ++i) amax = fmaxf(amax, fabsf(x[i]));
  const int s = mx_block_exp<FMT>(amax);
#pragma unroll
  for (int i = 0; i < 32; ++i) x[i] = ldexpf(x[i], -s);
  uint32_t w[8];
  mx_pack_block<FMT>(x, w);
  u32x4* d = (u32x4*)dst;
  d[0] = (u32x4){w[0], w[1], w[2], w[3]};
  if (FMT != 4) d[1] = (u32x4){w[4], w[5], w[6], w[7]};
  return (uint8_t)(s + 127);
}

// One thread per 32-element block of the rows of src [rows, K].
template <int FMT, typename TIN>
__global__ __launch_bounds__(256) void mx_quant_rows(const TIN* __restrict__ src, int rows,
                                                     int K, uint8_t* __restrict__ codes,
                                                     uint8_t* __restrict__ scales) {
  const int nb = K / 32;
  const size_t g = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (size_t)rows * nb) return;
  const size_t r = g / nb;
  const int b = (int)(g - r * nb);
  float x[32];
  const TIN* p = src + r * K + (size_t)b * 32;
#pragma unroll
  for (int i = 0; i < 32; ++i) x[i] = (float)p[i];
  scales[g] = mx_quant_block<FMT>(x, codes + r * mx_row_bytes(FMT, K) + mx_row_bytes(FMT, 32) * b);
}

// ------------------------------------------- MX grouped GEMM, 256 x 256
// The 8-wavefront 256 x 256 tile of gemm_bf16_wide (same tile order, DMA,
// swizzled 128-byte LDS rows, SwiGLU pairing), reading one 128-byte row
// segment per stage: 128 K (e4m3, padded e2m3) or 256 K (e2m1).  Per stage
// and 32x32 tile, v_mfma_scale_f32_32x32x64_f8f6f4 steps through K in
// 64-element slices with the two operands' E8M0 block scales as its scale
// operands, so the block scaling costs nothing beyond loading the scale
// bytes.  Lane (row r, half h) of a slice holds: e4m3 bytes 16h..16h+15 of
// each of the slice's two blocks; e2m3 / e2m1 all of block h; it supplies
// the scale of block h of its row (the instruction takes each block's
// scale from the lane of that row and half).  For e2m1, K % 256 == 128
// leaves a last stage of 128 K: its upper row halves are never loaded nor
// used.  SwiGLU epilogue: h = silu(A) * B rounded to BF16 in the LDS tile,
// then quantised per 32-column block straight to h codes and scale bytes.
template <int FMT, int EPI, bool GATHER>
__global__ __launch_bounds__(64 * XW, 1) void gemm_mx_wide(
    const uint8_t* __restrict__ A, const uint8_t* __restrict__ As,
    const int32_t* __restrict__ row_map, int T, const uint8_t* __restrict__ B,
    const uint8_t* __restrict__ Bs, void* __restrict__ Cv, uint8_t* __restrict__ Cscale,
    const int32_t* __restrict__ offsets, const int32_t* __restrict__ tile_start, int E, int N,
    int K, int f, int Ncols, int n_tiles, int grid_total) {
  typedef __attribute__((address_space(3))) void lds_void;
  constexpr bool PAIRED = EPI == EPI_SWIGLU;
  constexpr int KPS = FMT == 4 ? 256 : 128;  // K elements per stage
  constexpr int KK = KPS / 64;               // 64-K slices per stage
  constexpr int BPS = KPS / 32;              // scale blocks per stage
  __shared__ __attribute__((aligned(1024))) char lds[XLDS];
  const int b = blockIdx.x;
  const int Lt = xcd_tile(tile_start, E, n_tiles, grid_total, b);
  int e, row0, rows, nt;
  if (!find_tile_grouped(tile_start, offsets, E, GBM, N, n_tiles, Lt, e, row0, rows, nt)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 2, wn = wv & 3;
  const int n0 = nt * (PAIRED ? 128 : 256);
  const size_t Brows_e = PAIRED ? (size_t)2 * f : (size_t)Ncols;
  const size_t RB = mx_row_bytes(FMT, K);  // bytes of an operand row
  const int nbk = K / 32;                  // scale bytes of an operand row
  const uint8_t* asrc[XA_INS];
  const uint8_t* bsrc[XB_INS];
  bool a_lo[XA_INS], b_lo[XB_INS];  // the lane's chunk lies in the first 64 bytes
#pragma unroll
  for (int i = 0; i < XA_INS; ++i) {
    const int R = wv * (GBM / XW) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    const int r = row0 + min(R, rows - 1);
    const size_t arow = GATHER ? (size_t)min(max(row_map[r], 0), T - 1) : (size_t)r;
    asrc[i] = A + arow * RB + c * 16;
    a_lo[i] = c < 4;
  }
#pragma unroll
  for (int i = 0; i < XB_INS; ++i) {
    const int R = wv * (XBN / XW) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    const int wrow = PAIRED ? (R < 128 ? n0 + R : f + n0 + (R - 128)) : n0 + R;
    bsrc[i] = B + ((size_t)e * Brows_e + wrow) * RB + c * 16;
    b_lo[i] = c < 4;
  }
  const int fr = lane & 31, fh = lane >> 5;
  int aoff[4], asw[4], boff[2], bsw[2];
  const uint8_t* sarow[4];
  const uint8_t* sbrow[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int R = wm * 128 + i * 32 + fr;
    aoff[i] = R * 128;
    asw[i] = (R >> 1) & 7;
    const int r = row0 + min(R, rows - 1);
    const size_t arow = GATHER ? (size_t)min(max(row_map[r], 0), T - 1) : (size_t)r;
    sarow[i] = As + arow * nbk;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int R = (PAIRED ? (j == 0 ? wn * 32 : 128 + wn * 32) : wn * 64 + j * 32) + fr;
    boff[j] = XSTAGE_A + R * 128;
    bsw[j] = (R >> 1) & 7;
    const int wrow = PAIRED ? (R < 128 ? n0 + R : f + n0 + (R - 128)) : n0 + R;
    sbrow[j] = Bs + ((size_t)e * Brows_e + wrow) * nbk;
  }
  f32x16 acc[4][2];
  zero_acc(acc);
  const int nk = (K + KPS - 1) / KPS;
  const bool tail = K % KPS != 0;  // e2m1 only: last stage of 128 K
#define MX_ISSUE(kstep)                                                                        \
  {                                                                                            \
    char* st_ = lds + ((kstep) & 1) * XSTAGE;                                                  \
    const size_t k0_ = (size_t)(kstep) * 128;                                                  \
    const bool half_ = tail && (kstep) == nk - 1;                                              \
    _Pragma("unroll") for (int i = 0; i < XA_INS; ++i) if (!half_ || a_lo[i])                  \
        __builtin_amdgcn_global_load_lds(asrc[i] + k0_,                                        \
                                         (lds_void*)(st_ + (wv * (GBM / XW) + i * 8) * 128),   \
                                         16, 0, 0);                                            \
    _Pragma("unroll") for (int i = 0; i < XB_INS; ++i) if (!half_ || b_lo[i])                  \
        __builtin_amdgcn_global_load_lds(                                                      \
            bsrc[i] + k0_, (lds_void*)(st_ + XSTAGE_A + (wv * (XBN / XW) + i * 8) * 128), 16,  \
            0, 0);                                                                             \
  }
  // scale words of a stage: bytes [kstep * BPS, +BPS) of each row, loaded
  // one stage ahead into san / sbn
  uint32_t sa[4][BPS / 4], sb[2][BPS / 4], san[4][BPS / 4], sbn[2][BPS / 4];
#define MX_SCALES(SA, SB, kstep)                                                   \
  {                                                                                \
    const int o_ = (kstep) * BPS;                                                  \
    const bool half_ = tail && (kstep) == nk - 1;                                  \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) _Pragma("unroll") for (          \
        int w = 0; w < BPS / 4; ++w) SA[i][w] =                                    \
        (w == 0 || !half_) ? *(const uint32_t*)(sarow[i] + o_ + 4 * w) : 0u;       \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) _Pragma("unroll") for (          \
        int w = 0; w < BPS / 4; ++w) SB[j][w] =                                    \
        (w == 0 || !half_) ? *(const uint32_t*)(sbrow[j] + o_ + 4 * w) : 0u;       \
  }
  // fragment of slice kk for a row at LDS offset off with swizzle sw
#define MX_FRAG(out, off, sw, kk)                                                  \
  {                                                                                \
    const char* st_ = lds + (kt & 1) * XSTAGE;                                     \
    if (FMT == 0) {                                                                \
      const u32x4 lo_ = *(const u32x4*)(st_ + (off) + (((4 * (kk) + fh) ^ (sw)) << 4));     \
      const u32x4 hi_ = *(const u32x4*)(st_ + (off) + (((4 * (kk) + 2 + fh) ^ (sw)) << 4)); \
      out = (i32x8){(int)lo_[0], (int)lo_[1], (int)lo_[2], (int)lo_[3],            \
                    (int)hi_[0], (int)hi_[1], (int)hi_[2], (int)hi_[3]};           \
    } else if (FMT == 2) {                                                         \
      const u32x4 lo_ = *(const u32x4*)(st_ + (off) + (((4 * (kk) + 2 * fh) ^ (sw)) << 4));     \
      const u32x4 hi_ = *(const u32x4*)(st_ + (off) + (((4 * (kk) + 2 * fh + 1) ^ (sw)) << 4)); \
      out = (i32x8){(int)lo_[0], (int)lo_[1], (int)lo_[2], (int)lo_[3],            \
                    (int)hi_[0], (int)hi_[1], 0, 0};                               \
    } else {                                                                       \
      const u32x4 lo_ = *(const u32x4*)(st_ + (off) + (((2 * (kk) + fh) ^ (sw)) << 4)); \
      out = (i32x8){(int)lo_[0], (int)lo_[1], (int)lo_[2], (int)lo_[3], 0, 0, 0, 0}; \
    }                                                                              \
  }
  MX_ISSUE(0);
  if (nk > 1) {
    MX_ISSUE(1);
    WAIT_VM_LGKM0(XA_INS + XB_INS);
  } else {
    WAIT_VM_LGKM0(0);
  }
  MX_SCALES(sa, sb, 0);
  stage_barrier();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) MX_SCALES(san, sbn, kt + 1);
    const int kkn = (tail && kt == nk - 1) ? KK / 2 : KK;
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      if (kk < kkn) {
        i32x8 af[4], bfr[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) MX_FRAG(af[i], aoff[i], asw[i], kk);
#pragma unroll
        for (int j = 0; j < 2; ++j) MX_FRAG(bfr[j], boff[j], bsw[j], kk);
        const int blk = 2 * kk + fh, wsel = blk >> 2, sh = 8 * (blk & 3);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int sca = (int)((sa[i][wsel] >> sh) & 0xFFu);
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int scb = (int)((sb[j][wsel] >> sh) & 0xFFu);
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                bfr[j], af[i], acc[i][j], FMT, FMT, 0, scb, 0, sca);
          }
        }
      }
    }
    if (kt + 1 < nk) {
      WAIT_VM_LGKM0(0);
      stage_barrier();
      if (kt + 2 < nk) MX_ISSUE(kt + 2);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int w = 0; w < BPS / 4; ++w) sa[i][w] = san[i][w];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int w = 0; w < BPS / 4; ++w) sb[j][w] = sbn[j][w];
    }
  }
#undef MX_ISSUE
#undef MX_SCALES
#undef MX_FRAG
  WAIT_VM_LGKM0(0);
  stage_barrier();

  constexpr int CS = EPI == EPI_SWIGLU ? 128 : 256;
  constexpr int CLD = CS + 8;
  bf16_t* Cs = (bf16_t*)lds;
  const int cbase = fh * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rl = wm * 128 + i * 32 + fr;
#pragma unroll
    for (int j = 0; j < (EPI == EPI_SWIGLU ? 1 : 2); ++j) {
      const int col0 = EPI == EPI_SWIGLU ? wn * 32 : wn * 64 + j * 32;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        bf16x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float x = acc[i][j][g * 4 + q];
          if (EPI == EPI_SWIGLU) v[q] = (bf16_t)(silu(x) * acc[i][1][g * 4 + q]);
          else v[q] = (bf16_t)x;
        }
        *(bf16x4*)(Cs + rl * CLD + col0 + g * 8 + cbase) = v;
      }
    }
  }
  __syncthreads();
  if (EPI == EPI_SWIGLU) {
    // h codes [N, row bytes of f] and scale bytes [N, f/32]
    uint8_t* hc = (uint8_t*)Cv;
    const size_t RBf = mx_row_bytes(FMT, f);
    for (int c = tid; c < GBM * 4; c += 64 * XW) {
      const int rr = c >> 2, qb = c & 3;
      if (rr >= rows) continue;
      float x[32];
      const bf16_t* src = Cs + rr * CLD + qb * 32;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bf16x8 v = *(const bf16x8*)(src + 8 * q);
#pragma unroll
        for (int u = 0; u < 8; ++u) x[8 * q + u] = (float)v[u];
      }
      const size_t row = (size_t)(row0 + rr);
      const int blk = nt * 4 + qb;
      Cscale[row * (f / 32) + blk] =
          mx_quant_block<FMT>(x, hc + row * RBf + mx_row_bytes(FMT, 32) * blk);
    }
  } else {
    bf16_t* C = (bf16_t*)Cv;
    constexpr int CPR = CS / 8;
    for (int c = tid; c < GBM * CPR; c += 64 * XW) {
      const int rr = c / CPR, cc = (c - rr * CPR) * 8;
      if (rr >= rows) continue;
      *(u32x4*)(C + (size_t)(row0 + rr) * Ncols + (size_t)nt * CS + cc) =
          *(const u32x4*)(Cs + rr * CLD + cc);
    }
  }
}

#define MOE_INST_MX(FMT)                                                                      \
  template __global__ void gemm_mx_wide<FMT, EPI_SWIGLU, true>(                              \
      const uint8_t* __restrict__, const uint8_t* __restrict__, const int32_t* __restrict__, \
      int, const uint8_t* __restrict__, const uint8_t* __restrict__, void* __restrict__,     \
      uint8_t* __restrict__, const int32_t* __restrict__, const int32_t* __restrict__, int,  \
      int, int, int, int, int, int);                                                         \
  template __global__ void gemm_mx_wide<FMT, EPI_PLAIN, false>(                              \
      const uint8_t* __restrict__, const uint8_t* __restrict__, const int32_t* __restrict__, \
      int, const uint8_t* __restrict__, const uint8_t* __restrict__, void* __restrict__,     \
      uint8_t* __restrict__, const int32_t* __restrict__, const int32_t* __restrict__, int,  \
      int, int, int, int, int, int);
MOE_INST_MX(0)
MOE_INST_MX(2)
MOE_INST_MX(4)
#undef MOE_INST_MX

// ------------------------------------------------------------- backward
// Backward of the expert FFN for the rows of each expert (dY = w * dOut in
// slot order, supplied by the combine backward):
//   [A|B] = Xp W13^T  (gemm_bf16_wide<EPI_AB, gather>; or the forward's,
//                      stored by gemm_bf16_wide<EPI_SWIGLU_AB, gather>)
//   U = dY W2 (BF16)  (gemm_bf16_wide_bkm reading W2 K-major; on W2^T with
//                      the 256 x 128 tile when d_ff % 256 != 0)
//   h = silu(A) B, dA = U B silu'(A), dB = U silu(A)
//                     (dgrad_elem, reading U and [A|B])
//   dX_perm = [dA|dB] W13          (gemm_bf16_wide_bkm reading W13 K-major)
//   dW13_e = [dA|dB]^T Xp,  dW2_e = dY^T h          (gemm_wgrad_wide)
// The weight gradients are "NT" products with both operands contiguous
// along the reduction: the activations they reduce over are written
// transposed [channel][slot] with each expert's slot range padded to a
// multiple of PADK with zeros.

// Four consecutive weight-gradient values: FP32, or rounded to BF16.
__device__ __forceinline__ void store4(float* p, float a, float b, float c, float d) {
  *(f32x4*)p = (f32x4){a, b, c, d};
}
__device__ __forceinline__ void store4(bf16_t* p, float a, float b, float c, float d) {
  *(bf16x4*)p = (bf16x4){(bf16_t)a, (bf16_t)b, (bf16_t)c, (bf16_t)d};
}

// Slot ranges of the transposed buffers are padded per expert to a multiple
// of PADK (one K stage of the 256 x 256 weight-gradient tile).
constexpr int PADK = 64;

// dA, dB and h from U = dY W2 (BF16) and the recomputed [A|B], one block per
// 64 slot rows of one expert (tile_start of 64-row tiles) and 64 columns of
// f: dA and dB are stored row-major into [dA|dB] and, like h, transposed
// through LDS into the slot-major buffers at the expert's padded slot
// offset.  silu(a) = a s, s = 1/(1+exp(-a)); dA = U B (s + a s (1 - s)),
// dB = U a s, h = a s B.
constexpr int DE_TILE = 64;

__global__ __launch_bounds__(256) void dgrad_elem(
    const bf16_t* __restrict__ U, const bf16_t* __restrict__ AB, bf16_t* __restrict__ dAB,
    bf16_t* __restrict__ dABT, bf16_t* __restrict__ hT, int ldT,
    const int32_t* __restrict__ offsets, const int32_t* __restrict__ tile64,
    const int32_t* __restrict__ ptile, int E, int N, int f) {
  __shared__ __attribute__((aligned(16))) bf16_t Ls[3][DE_TILE][DE_TILE + 8];
  int e, row0, rows;
  if (!find_tile(tile64, offsets, E, DE_TILE, N, blockIdx.x, e, row0, rows)) return;
  const int n0 = blockIdx.y * DE_TILE, tid = threadIdx.x;
  const size_t ld2f = (size_t)2 * f;
  for (int it = tid; it < DE_TILE * (DE_TILE / 8); it += 256) {
    const int r = it >> 3, c8 = (it & 7) * 8;
    bf16x8 oa, ob, oh;
    if (r < rows) {
      const size_t row = (size_t)(row0 + r);
      const bf16x8 u = *(const bf16x8*)(U + row * f + n0 + c8);
      const bf16x8 av = *(const bf16x8*)(AB + row * ld2f + n0 + c8);
      const bf16x8 bv = *(const bf16x8*)(AB + row * ld2f + f + n0 + c8);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float uu = (float)u[q], a = (float)av[q], bb = (float)bv[q];
        const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-a));
        const float sa = a * sg;
        oa[q] = (bf16_t)(uu * bb * (sg + sa * (1.0f - sg)));
        ob[q] = (bf16_t)(uu * sa);
        oh[q] = (bf16_t)(sa * bb);
      }
      *(bf16x8*)(dAB + row * ld2f + n0 + c8) = oa;
      *(bf16x8*)(dAB + row * ld2f + f + n0 + c8) = ob;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) oa[q] = ob[q] = oh[q] = (bf16_t)0.0f;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      Ls[0][c8 + q][r] = oa[q];
      Ls[1][c8 + q][r] = ob[q];
      Ls[2][c8 + q][r] = oh[q];
    }
  }
  __syncthreads();
  const size_t pcol0 = (size_t)ptile[e] * PADK + (size_t)(row0 - offsets[e]);
  for (int it = tid; it < 3 * DE_TILE * (DE_TILE / 8); it += 256) {
    const int q = it / (DE_TILE * (DE_TILE / 8));
    const int rem = it - q * DE_TILE * (DE_TILE / 8);
    const int c = rem >> 3, r8 = (rem & 7) * 8;
    if (r8 >= rows) continue;
    bf16_t* dst = q == 2 ? hT + (size_t)(n0 + c) * ldT
                         : dABT + ((size_t)(q == 1 ? f : 0) + n0 + c) * ldT;
    *(u32x4*)(dst + pcol0 + r8) = *(const u32x4*)&Ls[q][c][r8];
  }
}

// Weight gradient of one expert: out_e[m][n] = sum over the expert's padded
// slot range of At[m][k] * Bt[n][k] (both [rows][ldT], contiguous along k;
// pads are zero).  Tile 256 x 128, FP32 results stored directly.
template <typename TO>
__global__ __launch_bounds__(256, 2) void gemm_wgrad(const bf16_t* __restrict__ At,
                                                     const bf16_t* __restrict__ Bt, int ldT,
                                                     const int32_t* __restrict__ ptile, int E,
                                                     int M, int Nn, TO* __restrict__ out,
                                                     int m_tiles, int n_tiles, int grid_total) {
  __shared__ __attribute__((aligned(1024))) char lds[DMA_LDS];
  const int b = blockIdx.x;
  const int per = grid_total >> 3;
  const int Lt = (b & 7) * per + (b >> 3);
  const int tiles_e = m_tiles * n_tiles;
  if (Lt >= E * tiles_e) return;
  const int e = Lt / tiles_e, rem = Lt - e * tiles_e;
  const int mt = rem / n_tiles, nt = rem - mt * n_tiles;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const size_t k0 = (size_t)ptile[e] * PADK;
  const int nk = (ptile[e + 1] - ptile[e]) * (PADK / GBK);
  const bf16_t* asrc[A_INS];
  const bf16_t* bsrc[B_INS];
#pragma unroll
  for (int i = 0; i < A_INS; ++i) {
    const int R = wv * (GBM / 4) + i * 16 + (lane >> 2);
    const int c = (lane & 3) ^ swz(R);
    asrc[i] = At + (size_t)(mt * GBM + R) * ldT + k0 + c * 8;
  }
#pragma unroll
  for (int i = 0; i < B_INS; ++i) {
    const int R = wv * (GBN / 4) + i * 16 + (lane >> 2);
    const int c = (lane & 3) ^ swz(R);
    bsrc[i] = Bt + (size_t)(nt * GBN + R) * ldT + k0 + c * 8;
  }
  int aoff[4], asw[4], boff[2], bsw[2];
  frag_offsets(wm, wn * 64, wn * 64 + 32, lane, aoff, asw, boff, bsw);
  f32x16 acc[4][2];
  zero_acc(acc);
  mma_pipeline<A_INS, B_INS>(lds, asrc, bsrc, nk, wv, lane, aoff, asw, boff, bsw, acc);
  const int fr = lane & 31, cbase = (lane >> 5) * 4;
  TO* oe = out + (size_t)e * M * Nn;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const size_t m = (size_t)mt * GBM + wm * 128 + i * 32 + fr;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int n = nt * GBN + wn * 64 + j * 32 + g * 8 + cbase;
        store4(oe + m * Nn + n, acc[i][j][g * 4], acc[i][j][g * 4 + 1], acc[i][j][g * 4 + 2],
               acc[i][j][g * 4 + 3]);
      }
  }
}

// Weight gradient on the 256 x 256 tile of gemm_bf16_wide (8 wavefronts,
// K = 64 per stage, two 64 KB stages): out_e[m][n] = sum over the expert's
// padded slot range of At[m][k] * Bt[n][k], FP32 results stored directly.
// M and Nn are multiples of 256; an expert without slots stores zeros.
template <typename TO>
__global__ __launch_bounds__(64 * XW, 1) void gemm_wgrad_wide(
    const bf16_t* __restrict__ At, const bf16_t* __restrict__ Bt, int ldT,
    const int32_t* __restrict__ ptile, int E, int M, int Nn, TO* __restrict__ out,
    int m_tiles, int n_tiles, int grid_total) {
  typedef __attribute__((address_space(3))) void lds_void;
  __shared__ __attribute__((aligned(1024))) char lds[2 * XSTAGE];
  const int b = blockIdx.x;
  const int per = grid_total >> 3;
  const int Lt = (b & 7) * per + (b >> 3);
  const int tiles_e = m_tiles * n_tiles;
  if (Lt >= E * tiles_e) return;
  const int e = Lt / tiles_e, rem = Lt - e * tiles_e;
  const int mt = rem / n_tiles, nt = rem - mt * n_tiles;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 2, wn = wv & 3;
  const size_t k0 = (size_t)ptile[e] * PADK;
  const int nk = (ptile[e + 1] - ptile[e]) * (PADK / XBK);
  const bf16_t* asrc[XA_INS];
  const bf16_t* bsrc[XB_INS];
#pragma unroll
  for (int i = 0; i < XA_INS; ++i) {
    const int R = wv * (GBM / XW) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    asrc[i] = At + (size_t)(mt * GBM + R) * ldT + k0 + c * 8;
  }
#pragma unroll
  for (int i = 0; i < XB_INS; ++i) {
    const int R = wv * (XBN / XW) + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((R >> 1) & 7);
    bsrc[i] = Bt + (size_t)(nt * XBN + R) * ldT + k0 + c * 8;
  }
  const int fr = lane & 31, fh = lane >> 5;
  int aoff[4], asw[4], boff[2], bsw[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int R = wm * 128 + i * 32 + fr;
    aoff[i] = R * 128;
    asw[i] = (R >> 1) & 7;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int R = wn * 64 + j * 32 + fr;
    boff[j] = XSTAGE_A + R * 128;
    bsw[j] = (R >> 1) & 7;
  }
  f32x16 acc[4][2];
  zero_acc(acc);
#define W_ISSUE(kstep)                                                                         \
  {                                                                                            \
    char* st_ = lds + ((kstep) & 1) * XSTAGE;                                                  \
    const int k0_ = (kstep) * XBK;                                                             \
    _Pragma("unroll") for (int i = 0; i < XA_INS; ++i) __builtin_amdgcn_global_load_lds(       \
        asrc[i] + k0_, (lds_void*)(st_ + (wv * (GBM / XW) + i * 8) * 128), 16, 0, 0);          \
    _Pragma("unroll") for (int i = 0; i < XB_INS; ++i) __builtin_amdgcn_global_load_lds(       \
        bsrc[i] + k0_, (lds_void*)(st_ + XSTAGE_A + (wv * (XBN / XW) + i * 8) * 128), 16, 0,   \
        0);                                                                                    \
  }
#define W_READ(AF, BF, stp, ks)                                                          \
  {                                                                                      \
    const char* st_ = lds + ((stp) & 1) * XSTAGE;                                        \
    const int c_ = (ks) * 2 + fh;                                                        \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) AF[i] =                                \
        *(const bf16x8*)(st_ + aoff[i] + ((c_ ^ asw[i]) << 4));                          \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) BF[j] =                                \
        *(const bf16x8*)(st_ + boff[j] + ((c_ ^ bsw[j]) << 4));                          \
  }
#define W_MFMA(AF, BF)                                                                   \
  _Pragma("unroll") for (int i = 0; i < 4; ++i) _Pragma("unroll") for (int j = 0; j < 2; \
                                                                       ++j) acc[i][j] =  \
      __builtin_amdgcn_mfma_f32_32x32x16_bf16(BF[j], AF[i], acc[i][j], 0, 0, 0);
  if (nk > 0) {
    bf16x8 a0[4], b0[2], a1[4], b1[2];
    W_ISSUE(0);
    if (nk > 1) {
      W_ISSUE(1);
      WAIT_VM_LGKM0(XA_INS + XB_INS);
    } else {
      WAIT_VM_LGKM0(0);
    }
    stage_barrier();
    W_READ(a0, b0, 0, 0);
    for (int kt = 0; kt < nk; ++kt) {
      __builtin_amdgcn_iglp_opt(1);
      W_READ(a1, b1, kt, 1);
      W_MFMA(a0, b0);
      W_READ(a0, b0, kt, 2);
      W_MFMA(a1, b1);
      W_READ(a1, b1, kt, 3);
      W_MFMA(a0, b0);
      WAIT_VM_LGKM0(0);
      stage_barrier();
      if (kt + 2 < nk) W_ISSUE(kt + 2);
      if (kt + 1 < nk) W_READ(a0, b0, kt + 1, 0);
      W_MFMA(a1, b1);
    }
  }
#undef W_ISSUE
#undef W_READ
#undef W_MFMA
  const int cbase = fh * 4;
  TO* oe = out + (size_t)e * M * Nn;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const size_t m = (size_t)mt * GBM + wm * 128 + i * 32 + fr;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int n = nt * XBN + wn * 64 + j * 32 + g * 8 + cbase;
        store4(oe + m * Nn + n, acc[i][j][g * 4], acc[i][j][g * 4 + 1], acc[i][j][g * 4 + 2],
               acc[i][j][g * 4 + 3]);
      }
  }
}

#define MOE_INST_WG(TO)                                                                      \
  template __global__ void gemm_wgrad<TO>(const bf16_t* __restrict__, const bf16_t* __restrict__, \
                                          int, const int32_t* __restrict__, int, int, int,     \
                                          TO* __restrict__, int, int, int);                    \
  template __global__ void gemm_wgrad_wide<TO>(const bf16_t* __restrict__,                     \
                                               const bf16_t* __restrict__, int,                \
                                               const int32_t* __restrict__, int, int, int,     \
                                               TO* __restrict__, int, int, int);
MOE_INST_WG(float)
MOE_INST_WG(bf16_t)
#undef MOE_INST_WG

// out[b][c][r] = in[b][r][c], 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void batched_transpose(const bf16_t* __restrict__ in,
                                                         bf16_t* __restrict__ out, int R, int C) {
  // 64 x 64 tiles, 16-byte loads along C and 16-byte stores along R (R and
  // C are multiples of 64)
  __shared__ __attribute__((aligned(16))) bf16_t tile[64][72];
  const size_t base = (size_t)blockIdx.z * R * C;
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  for (int v = threadIdx.x; v < 512; v += 256) {
    const int r = v >> 3, cc = (v & 7) * 8;
    *(bf16x8*)&tile[r][cc] = *(const bf16x8*)(in + base + (size_t)(r0 + r) * C + c0 + cc);
  }
  __syncthreads();
  for (int v = threadIdx.x; v < 512; v += 256) {
    const int c = v >> 3, rr = (v & 7) * 8;
    bf16x8 y;
#pragma unroll
    for (int u = 0; u < 8; ++u) y[u] = tile[rr + u][c];
    *(bf16x8*)(out + base + (size_t)(c0 + c) * R + r0 + rr) = y;
  }
}
// Channels per block of slot_transpose: ST_CH chunks of 64, all loaded
// before the transposed stores, so the slot lookup (a search over the
// expert tiles) is shared by them and their loads are in flight together.
constexpr int ST_CH = 4;
__global__ __launch_bounds__(256) void slot_transpose(const bf16_t* __restrict__ src,
                                                      const int32_t* __restrict__ row_map, int T,
                                                      int C, const int32_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ ptile, int E,
                                                      bf16_t* __restrict__ outT, int ldT) {
  // 64 padded slots x ST_CH * 64 channels per block; 16-byte loads of
  // token rows, 16-byte stores along the slots (C, ldT and the slot offset
  // are multiples of 64)
  __shared__ __attribute__((aligned(16))) bf16_t tile[ST_CH][64][72];
  __shared__ int srow[64];
  __shared__ int sp[MOE_MAX_E + 1];
  const int tid = threadIdx.x;
  const int p0 = blockIdx.x * 64, cb = blockIdx.y * 64 * ST_CH;
  const int total = ptile[E] * PADK;
  if (p0 >= total) return;
  for (int i = tid; i <= E; i += 256) sp[i] = ptile[i];
  __syncthreads();
  if (tid < 64) {
    const int p = p0 + tid;
    int r = -1;
    if (p < total) {
      int lo = 0, hi = E - 1;  // largest e with pad_off[e] <= p
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sp[mid] * PADK <= p) lo = mid;
        else hi = mid - 1;
      }
      const int i = p - sp[lo] * PADK;
      if (i < offsets[lo + 1] - offsets[lo]) {
        r = offsets[lo] + i;
        if (row_map) r = min(max(row_map[r], 0), T - 1);
      }
    }
    srow[tid] = r;
  }
  __syncthreads();
  const int nch = min(ST_CH, (C - cb) / 64);
  bf16x8 x[ST_CH][2];
#pragma unroll
  for (int q = 0; q < ST_CH; ++q)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int v = tid + 256 * h, pl = v >> 3, cc = (v & 7) * 8;
      const int r = srow[pl];
      if (q < nch && r >= 0) {
        x[q][h] = *(const bf16x8*)(src + (size_t)r * C + cb + q * 64 + cc);
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) x[q][h][u] = (bf16_t)0.0f;
      }
    }
#pragma unroll
  for (int q = 0; q < ST_CH; ++q)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int v = tid + 256 * h, pl = v >> 3, cc = (v & 7) * 8;
      *(bf16x8*)&tile[q][pl][cc] = x[q][h];
    }
  __syncthreads();
  for (int q = 0; q < nch; ++q)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int v = tid + 256 * h, c = v >> 3, pr = (v & 7) * 8;
      if (p0 + pr >= total) continue;
      bf16x8 y;
#pragma unroll
      for (int u = 0; u < 8; ++u) y[u] = tile[q][pr + u][c];
      *(bf16x8*)(outT + (size_t)(cb + q * 64 + c) * ldT + p0 + pr) = y;
    }
}

// Zero each expert's pad columns [pad_off[e] + rows_e, pad_off[e+1]) of a
// transposed buffer with M rows.
__global__ __launch_bounds__(256) void pad_zero(bf16_t* __restrict__ buf, int M, int ldT,
                                                const int32_t* __restrict__ offsets,
                                                const int32_t* __restrict__ ptile) {
  const int e = blockIdx.x;
  const int m = blockIdx.y * 256 + threadIdx.x;
  if (m >= M) return;
  const int a = ptile[e] * PADK + (offsets[e + 1] - offsets[e]), z = ptile[e + 1] * PADK;
  for (int p = a; p < z; ++p) buf[(size_t)m * ldT + p] = (bf16_t)0.0f;
}

// ---------------------------------------------------------------- FP32 SIMT
// Block tile 64 rows x 64 B-rows, K step 16, 256 threads with 4 x 4 outputs.
// SwiGLU mode: B-rows 0..31 = W1 rows n0..n0+31, 32..63 = the W3 rows; a
// thread's column pair {2tx, 2tx+1} is taken from both halves.

constexpr int FBM = 64, FBK = 16;

template <bool SWIGLU>
__global__ __launch_bounds__(256) void gemm_f32(const float* __restrict__ A,
                                                const float* __restrict__ B, float* __restrict__ C,
                                                const int32_t* __restrict__ offsets,
                                                const int32_t* __restrict__ tile_start, int E,
                                                int N, int K, int f, int Ncols) {
  __shared__ float As[FBK][FBM + 1];
  __shared__ float Bs[FBK][64 + 1];
  int e, row0, rows;
  if (!find_tile(tile_start, offsets, E, FBM, N, blockIdx.x, e, row0, rows)) return;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int nspan = SWIGLU ? 32 : 64;
  const int n0 = blockIdx.y * nspan;
  const size_t Brows_e = SWIGLU ? (size_t)2 * f : (size_t)Ncols;
  const float* Be = B + (size_t)e * Brows_e * K;
  const int nlim = SWIGLU ? f : Ncols;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
  for (int k0 = 0; k0 < K; k0 += FBK) {
    for (int i = tid; i < FBM * FBK; i += 256) {
      const int r = i / FBK, c = i % FBK, kk = k0 + c;
      As[c][r] = (r < rows && kk < K) ? A[(size_t)(row0 + r) * K + kk] : 0.0f;
      int n = SWIGLU ? (r < 32 ? n0 + r : n0 + r - 32) : n0 + r;
      int src = SWIGLU ? (r < 32 ? n : f + n) : n;
      Bs[c][r] = (n < nlim && kk < K) ? Be[(size_t)src * K + kk] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < FBK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = SWIGLU ? (j < 2 ? tx * 2 + j : 32 + tx * 2 + (j - 2)) : tx * 4 + j;
        b[j] = Bs[kk][col];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rl = ty * 4 + i;
    if (rl >= rows) continue;
    const size_t row = (size_t)(row0 + rl);
    if (SWIGLU) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + tx * 2 + j;
        if (n < f) C[row * Ncols + n] = silu(acc[i][j]) * acc[i][j + 2];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + tx * 4 + j;
        if (n < Ncols) C[row * Ncols + n] = acc[i][j];
      }
    }
  }
}

struct FfnWs {
  int32_t* tile_start;
  int32_t* tile_start_big;
  void* h;      // h [N, f] in cfg.act; MX experts: h codes [N, row bytes of f]
  fp8_t* hq;    // FP8 path: codes of h [N, f]
  float* hs;    // FP8 path: scales of h [N, f/128]
  uint8_t* hx;  // MX experts: scale bytes of h [N, f/32]
};

// Matrix-instruction format selector of an MX dtype, -1 otherwise.
int mx_format(int dtype) {
  switch (dtype) {
    case MOE_MXFP8E4M3: return 0;
    case MOE_MXFP6E2M3: return 2;
    case MOE_MXFP4E2M1: return 4;
    default: return -1;
  }
}

FfnWs carve_ffn(const moe_cfg& c, void* base, size_t* total) {
  WsCarve wc{(char*)base, 0};
  FfnWs r;
  r.tile_start = wc.take<int32_t>((size_t)c.E + 1);
  r.tile_start_big = wc.take<int32_t>((size_t)c.E + 1);
  const size_t N = (size_t)c.T * c.k;
  const int mxf = mx_format(c.w);
  // FP8 experts keep h only as codes and scales (quantised by GEMM 1)
  r.h = wc.take<char>(mxf >= 0                ? N * mx_row_bytes(mxf, (size_t)c.d_ff)
                      : c.w == MOE_FP8E4M3 ? 0
                                           : N * (size_t)c.d_ff * act_bytes(c.act));
  r.hq = nullptr;
  r.hs = nullptr;
  r.hx = mxf >= 0 ? wc.take<uint8_t>(N * (size_t)(c.d_ff / 32)) : nullptr;
  if (c.w == MOE_FP8E4M3) {
    r.hq = wc.take<fp8_t>(N * (size_t)c.d_ff);
    r.hs = wc.take<float>(N * (size_t)(c.d_ff / 128));
  }
  if (total) *total = align_up(wc.off, 256);
  return r;
}

}  // namespace moe_gemm
using namespace moe_gemm;

size_t ffn_ws_bytes(const moe_cfg& c) {
  size_t total = 0;
  carve_ffn(c, nullptr, &total);
  return total;
}

namespace moe_gemm {

// The FP8 expert products: GEMM 1 + SwiGLU with the 1 x 128 quantisation
// of h in its epilogue (token rows gathered through row_map when it is
// given), GEMM 2.
void launch_fp8_ffn(const moe_cfg& c, const FfnWs& w, const fp8_t* Aq, const float* As,
                    const int32_t* row_map, const int32_t* offsets, const fp8_t* W13,
                    const float* W13_scale, const fp8_t* W2, const float* W2_scale, bf16_t* Y,
                    hipStream_t st) {
  const int N = c.T * c.k;
  hipLaunchKernelGGL(ffn_tiles, dim3(1), dim3(1024), 0, st, offsets, c.E, FQ_BM, w.tile_start);
  const int mt1 = (N + FQ_BM - 1) / FQ_BM + c.E;
  const int nt1 = c.d_ff / 128;
  const int G1 = (mt1 * nt1 + 7) / 8 * 8;
  // h leaves GEMM 1 as its 1 x 128 FP8 codes and scales
  PROF_BEGIN("gemm1_swiglu", st);
  if (row_map)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_fp8_q<true, false>), dim3(G1), dim3(64 * FQ_W), 0,
                       st, Aq, As, row_map, c.T, W13, W13_scale, w.hq, w.hs, nullptr, offsets,
                       w.tile_start, c.E, N, c.d, c.d_ff, nt1, G1);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_fp8_q<false, false>), dim3(G1), dim3(64 * FQ_W), 0,
                       st, Aq, As, nullptr, 0, W13, W13_scale, w.hq, w.hs, nullptr, offsets,
                       w.tile_start, c.E, N, c.d, c.d_ff, nt1, G1);
  PROF_END("gemm1_swiglu", st);
  PROF_BEGIN("gemm2", st);
  if (c.d % 256 == 0) {
    // 128 slot rows x 256 output columns per tile, the same tile schedule
    const int nt2 = c.d / 256;
    const int G2 = (mt1 * nt2 + 7) / 8 * 8;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_fp8_q<false, true>), dim3(G2), dim3(64 * FQ_W), 0,
                       st, (const fp8_t*)w.hq, (const float*)w.hs, nullptr, 0, W2, W2_scale,
                       nullptr, nullptr, Y, offsets, w.tile_start, c.E, N, c.d_ff, c.d, nt2, G2);
  } else {
    hipLaunchKernelGGL(ffn_tiles, dim3(1), dim3(1024), 0, st, offsets, c.E, GBM,
                       w.tile_start_big);
    const int mt_big = (N + GBM - 1) / GBM + c.E;
    const int nt2 = c.d / 128;
    const int G2 = (mt_big * nt2 + 7) / 8 * 8;
    hipLaunchKernelGGL(gemm_fp8_big, dim3(G2), dim3(256), 0, st, (const fp8_t*)w.hq,
                       (const float*)w.hs, W2, W2_scale, Y, offsets, w.tile_start_big, c.E, N,
                       c.d_ff, c.d, nt2, G2);
  }
  PROF_END("gemm2", st);
}

}  // namespace moe_gemm

extern "C" moe_status moe_expert_ffn(const moe_cfg* cfg, const void* X_perm,
                                     const float* X_perm_scale, const int32_t* offsets,
                                     const void* W13, const float* W13_scale, const void* W2,
                                     const float* W2_scale, void* Y, void* ws, size_t ws_bytes,
                                     void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (!offsets || !W13 || !W2) return MOE_EINVAL;
  if (c.T > 0 && (!X_perm || !Y)) return MOE_EINVAL;
  if (!aligned(X_perm, 16) || !aligned(W13, 16) || !aligned(W2, 16) || !aligned(Y, 16) ||
      !aligned(offsets, 4) || !aligned(X_perm_scale, 4) || !aligned(W13_scale, 4) ||
      !aligned(W2_scale, 4))
    return MOE_EINVAL;
  const bool f32path = c.act == MOE_F32 && c.w == MOE_F32;
  const bool bf16path = c.act == MOE_BF16 && c.w == MOE_BF16;
  const bool fp8path = c.act == MOE_BF16 && c.w == MOE_FP8E4M3;
  if (!f32path && !bf16path && !fp8path) return MOE_EUNSUPPORTED;
  if (bf16path && (c.d_ff % 64 != 0 || c.d % 128 != 0)) return MOE_EUNSUPPORTED;
  if (fp8path && (c.d_ff % 128 != 0 || c.d % 128 != 0)) return MOE_EUNSUPPORTED;
  if (fp8path && (!W13_scale || !W2_scale || (c.T > 0 && !X_perm_scale))) return MOE_EINVAL;
  if (ws_bytes < ffn_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  if (c.T == 0) return MOE_OK;
  hipStream_t st = (hipStream_t)stream;
  FfnWs w = carve_ffn(c, ws, nullptr);
  const int N = c.T * c.k;
  if (fp8path) {
    launch_fp8_ffn(c, w, (const fp8_t*)X_perm, X_perm_scale, nullptr, offsets, (const fp8_t*)W13,
                   W13_scale, (const fp8_t*)W2, W2_scale, (bf16_t*)Y, st);
  } else if (bf16path) {
    // 256-row tiles (d_ff % 64 == 0 and d % 128 == 0 were checked above):
    // 256 x 256 where d_ff % 128 (GEMM 1) or d % 256 (GEMM 2) allows it,
    // 256 x 128 otherwise
    hipLaunchKernelGGL(ffn_tiles, dim3(1), dim3(1024), 0, st, offsets, c.E, GBM, w.tile_start_big);
    const int mt_big = (N + GBM - 1) / GBM + c.E;
    PROF_BEGIN("gemm1_swiglu", st);
    if (c.d_ff % 128 == 0 && c.d % XBK == 0) {
      const int nt = c.d_ff / 128;
      const int G = (mt_big * nt + 7) / 8 * 8;
      hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_bf16_wide<EPI_SWIGLU, false>), dim3(G),
                         dim3(64 * XW), 0, st, (const bf16_t*)X_perm, nullptr, 0,
                         (const bf16_t*)W13, (bf16_t*)w.h, offsets, w.tile_start_big, c.E, N, c.d,
                         c.d_ff, c.d_ff, nt, G, nullptr);
    } else {
      const int nt = c.d_ff / 64;
      const int G = (mt_big * nt + 7) / 8 * 8;
      hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_bf16_big<EPI_SWIGLU, false>), dim3(G), dim3(256), 0,
                         st, (const bf16_t*)X_perm, nullptr, 0, (const bf16_t*)W13, (bf16_t*)w.h,
                         offsets, w.tile_start_big, c.E, N, c.d, c.d_ff, c.d_ff, nt, G);
    }
    PROF_END("gemm1_swiglu", st);
    PROF_BEGIN("gemm2", st);
    if (c.d % 256 == 0 && c.d_ff % XBK == 0) {
      const int nt = c.d / 256;
      const int G = (mt_big * nt + 7) / 8 * 8;
      hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_bf16_wide<EPI_PLAIN, false>), dim3(G),
                         dim3(64 * XW), 0, st, (const bf16_t*)w.h, nullptr, 0, (const bf16_t*)W2,
                         (bf16_t*)Y, offsets, w.tile_start_big, c.E, N, c.d_ff, c.d_ff, c.d, nt,
                         G, nullptr);
    } else {
      const int nt = c.d / 128;
      const int G = (mt_big * nt + 7) / 8 * 8;
      hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_bf16_big<EPI_PLAIN, false>), dim3(G), dim3(256), 0,
                         st, (const bf16_t*)w.h, nullptr, 0, (const bf16_t*)W2, (bf16_t*)Y, offsets,
                         w.tile_start_big, c.E, N, c.d_ff, c.d_ff, c.d, nt, G);
    }
    PROF_END("gemm2", st);
  } else {
    hipLaunchKernelGGL(ffn_tiles, dim3(1), dim3(1024), 0, st, offsets, c.E, FBM, w.tile_start);
    dim3 g1((N + FBM - 1) / FBM + c.E, (c.d_ff + 31) / 32);
    PROF_BEGIN("gemm1_swiglu", st);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_f32<true>), g1, dim3(256), 0, st, (const float*)X_perm,
                       (const float*)W13, (float*)w.h, offsets, w.tile_start, c.E, N, c.d, c.d_ff,
                       c.d_ff);
    PROF_END("gemm1_swiglu", st);
    dim3 g2((N + FBM - 1) / FBM + c.E, (c.d + 63) / 64);
    PROF_BEGIN("gemm2", st);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_f32<false>), g2, dim3(256), 0, st, (const float*)w.h,
                       (const float*)W2, (float*)Y, offsets, w.tile_start, c.E, N, c.d_ff, c.d_ff,
                       c.d);
    PROF_END("gemm2", st);
  }
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

namespace moe_gemm {

struct FfnBwdWs {
  int32_t* tile_start;
  int32_t* ptile;
  int32_t* tile64;  // schedule of 64-row tiles (the dA/dB/h pass)
  bf16_t *W2T, *AB, *U, *dAB, *dABT, *hT, *XpT, *dYT;
  int ldT;
};

// Row pitch of the transposed slot-major buffers: every expert's slot range
// padded to a multiple of PADK, rounded up to 64 elements.
int bwd_ldT(const moe_cfg& c) {
  const size_t N = (size_t)c.T * c.k;
  return (int)align_up(N + (size_t)PADK * c.E, 64);
}

FfnBwdWs carve_ffn_bwd(const moe_cfg& c, void* base, size_t* total) {
  WsCarve wc{(char*)base, 0};
  FfnBwdWs r;
  const size_t N = (size_t)c.T * c.k, d = c.d, f = c.d_ff, E = c.E;
  r.ldT = bwd_ldT(c);
  r.tile_start = wc.take<int32_t>(E + 1);
  r.ptile = wc.take<int32_t>(E + 1);
  r.tile64 = wc.take<int32_t>(E + 1);
  // W2 transposed only for the 256 x 128 tile of U (d_ff % 256 != 0); the
  // other data-gradient products read the weights K-major as stored
  r.W2T = f % XBN != 0 ? wc.take<bf16_t>(E * f * d) : nullptr;
  r.AB = wc.take<bf16_t>(N * 2 * f);
  r.U = wc.take<bf16_t>(N * f);
  r.dAB = wc.take<bf16_t>(N * 2 * f);
  r.dABT = wc.take<bf16_t>(2 * f * r.ldT);
  r.hT = wc.take<bf16_t>(f * r.ldT);
  r.XpT = wc.take<bf16_t>(d * r.ldT);
  r.dYT = wc.take<bf16_t>(d * r.ldT);
  if (total) *total = align_up(wc.off, 256);
  return r;
}

}  // namespace moe_gemm
using namespace moe_gemm;

size_t ffn_bwd_ws_bytes(const moe_cfg& c) {
  size_t total = 0;
  carve_ffn_bwd(c, nullptr, &total);
  return total;
}

namespace {

// The expert backward; AB (the forward's pre-activations) replaces the
// recomputation of [A|B] when given.
moe_status ffn_bwd_impl(const moe_cfg* cfg, const void* X, const int32_t* row_map,
                        const int32_t* offsets, const void* dY, const void* W13, const void* W2,
                        const void* AB, void* dX_perm, void* dW13, void* dW2, int grad_dtype,
                        void* ws, size_t ws_bytes, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.act != MOE_BF16 || c.w != MOE_BF16) return MOE_EUNSUPPORTED;
  if (c.d_ff % 128 != 0 || c.d % 256 != 0) return MOE_EUNSUPPORTED;
  if (grad_dtype != MOE_F32 && grad_dtype != MOE_BF16) return MOE_EINVAL;
  if (!offsets || !W13 || !W2 || !dW13 || !dW2) return MOE_EINVAL;
  if (c.T > 0 && (!X || !row_map || !dY || !dX_perm)) return MOE_EINVAL;
  if (!aligned(X, 16) || !aligned(dY, 16) || !aligned(W13, 16) || !aligned(W2, 16) ||
      !aligned(dX_perm, 16) || !aligned(dW13, 16) || !aligned(dW2, 16) || !aligned(offsets, 4) ||
      !aligned(row_map, 4) || !aligned(AB, 16))
    return MOE_EINVAL;
  if (ws_bytes < ffn_bwd_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  FfnBwdWs w = carve_ffn_bwd(c, ws, nullptr);
  const int N = c.T * c.k, d = c.d, f = c.d_ff, E = c.E;
  const bf16_t* Xb = (const bf16_t*)X;
  const bf16_t* dYb = (const bf16_t*)dY;
  PROF_BEGIN("ffn_bwd", st);
  hipLaunchKernelGGL(ffn_tiles, dim3(1), dim3(1024), 0, st, offsets, E, GBM, w.tile_start);
  hipLaunchKernelGGL(ffn_tiles, dim3(1), dim3(1024), 0, st, offsets, E, PADK, w.ptile);
  hipLaunchKernelGGL(ffn_tiles, dim3(1), dim3(1024), 0, st, offsets, E, DE_TILE, w.tile64);
  // the data-gradient products read W13 and W2 K-major as stored (no
  // transposed copy), except U on the 256 x 128 tile (d_ff % 256 != 0)
  if (f % XBN != 0)
    hipLaunchKernelGGL(batched_transpose, dim3(f / 64, d / 64, E), dim3(256), 0, st,
                       (const bf16_t*)W2, w.W2T, d, f);
  const int mt = (N + GBM - 1) / GBM + E;
  if (N > 0) {
    // [A|B] = Xp W13^T with the permute recomputed (f % 128 == 0), unless
    // the forward's are given
    const bf16_t* ABp = (const bf16_t*)AB;
    if (!ABp) {
      const int nt = f / 128, G = (mt * nt + 7) / 8 * 8;
      hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_bf16_wide<EPI_AB, true>), dim3(G), dim3(64 * XW), 0,
                         st, Xb, row_map, c.T, (const bf16_t*)W13, w.AB, offsets, w.tile_start, E,
                         N, d, f, 2 * f, nt, G, nullptr);
      ABp = w.AB;
    }
    {  // U = dY W2 (BF16, 256 columns of f per tile when f allows), then dA, dB, h
      if (f % XBN == 0) {
        const int nt = f / XBN, G = (mt * nt + 7) / 8 * 8;
        hipLaunchKernelGGL(gemm_bf16_wide_bkm, dim3(G), dim3(64 * XW), 0, st, dYb,
                           (const bf16_t*)W2, w.U, offsets, w.tile_start, E, N, d, f, nt, G);
      } else {
        const int nt = f / GBN, G = (mt * nt + 7) / 8 * 8;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_bf16_big<EPI_PLAIN, false>), dim3(G), dim3(256),
                           0, st, dYb, nullptr, 0, w.W2T, w.U, offsets, w.tile_start, E, N, d, d,
                           f, nt, G);
      }
      const int m64 = (N + DE_TILE - 1) / DE_TILE + E;
      hipLaunchKernelGGL(dgrad_elem, dim3(m64, f / DE_TILE), dim3(256), 0, st, w.U, ABp, w.dAB,
                         w.dABT, w.hT, w.ldT, offsets, w.tile64, w.ptile, E, N, f);
    }
    {  // dX_perm = [dA|dB] W13 (d % 256 == 0: the 256 x 256 tile, W13 K-major)
      const int nt = d / 256, G = (mt * nt + 7) / 8 * 8;
      hipLaunchKernelGGL(gemm_bf16_wide_bkm, dim3(G), dim3(64 * XW), 0, st, w.dAB,
                         (const bf16_t*)W13, (bf16_t*)dX_perm, offsets, w.tile_start, E, N,
                         2 * f, d, nt, G);
    }
    const int pblocks = (w.ldT + 63) / 64;
    const dim3 gst(pblocks, (d / 64 + ST_CH - 1) / ST_CH);
    hipLaunchKernelGGL(slot_transpose, gst, dim3(256), 0, st, Xb, row_map, c.T, d, offsets,
                       w.ptile, E, w.XpT, w.ldT);
    hipLaunchKernelGGL(slot_transpose, gst, dim3(256), 0, st, dYb, nullptr, N, d, offsets,
                       w.ptile, E, w.dYT, w.ldT);
    hipLaunchKernelGGL(pad_zero, dim3(E, (2 * f + 255) / 256), dim3(256), 0, st, w.dABT, 2 * f,
                       w.ldT, offsets, w.ptile);
    hipLaunchKernelGGL(pad_zero, dim3(E, (f + 255) / 256), dim3(256), 0, st, w.hT, f, w.ldT,
                       offsets, w.ptile);
  }
  {  // dW13_e = [dA|dB]^T Xp (M = 2f, N = d); dW2_e = dY^T h (M = d, N = f);
     // the 256 x 256 tile where the output width is a multiple of 256
    const int m1 = 2 * f / GBM, n1 = d / XBN;  // d % 256 == 0 was checked
    const int G1 = (E * m1 * n1 + 7) / 8 * 8;
    const int m2 = d / GBM;
    const bool wide2 = f % XBN == 0;
    const int n2 = wide2 ? f / XBN : f / GBN;
    const int G2 = (E * m2 * n2 + 7) / 8 * 8;
#define WGRAD(TO)                                                                              \
  {                                                                                            \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_wgrad_wide<TO>), dim3(G1), dim3(64 * XW), 0, st,   \
                       w.dABT, w.XpT, w.ldT, w.ptile, E, 2 * f, d, (TO*)dW13, m1, n1, G1);     \
    if (wide2)                                                                                 \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_wgrad_wide<TO>), dim3(G2), dim3(64 * XW), 0, st, \
                         w.dYT, w.hT, w.ldT, w.ptile, E, d, f, (TO*)dW2, m2, n2, G2);          \
    else                                                                                       \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_wgrad<TO>), dim3(G2), dim3(256), 0, st, w.dYT,   \
                         w.hT, w.ldT, w.ptile, E, d, f, (TO*)dW2, m2, n2, G2);                 \
  }
    if (grad_dtype == MOE_BF16) WGRAD(bf16_t)
    else WGRAD(float)
#undef WGRAD
  }
  PROF_END("ffn_bwd", st);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

}  // namespace

extern "C" moe_status moe_expert_ffn_bwd(const moe_cfg* cfg, const void* X,
                                         const int32_t* row_map, const int32_t* offsets,
                                         const void* dY, const void* W13, const void* W2,
                                         void* dX_perm, void* dW13, void* dW2, int grad_dtype,
                                         void* ws, size_t ws_bytes, void* stream) {
  return ffn_bwd_impl(cfg, X, row_map, offsets, dY, W13, W2, nullptr, dX_perm, dW13, dW2,
                      grad_dtype, ws, ws_bytes, stream);
}

extern "C" moe_status moe_expert_ffn_bwd_saved(const moe_cfg* cfg, const void* X,
                                               const int32_t* row_map, const int32_t* offsets,
                                               const void* dY, const void* W13, const void* W2,
                                               const void* AB, void* dX_perm, void* dW13,
                                               void* dW2, int grad_dtype, void* ws,
                                               size_t ws_bytes, void* stream) {
  if (cfg && cfg->T > 0 && !AB) return MOE_EINVAL;
  return ffn_bwd_impl(cfg, X, row_map, offsets, dY, W13, W2, AB, dX_perm, dW13, dW2, grad_dtype,
                      ws, ws_bytes, stream);
}

extern "C" moe_status moe_quantize_fp8(int rows, int cols, int block_rows, int src_dtype,
                                       const void* src, uint8_t* codes, float* scales,
                                       void* stream) {
  if (rows < 0 || cols < 0 || cols % 128 != 0) return MOE_EINVAL;
  if (block_rows != 1 && block_rows != 128) return MOE_EINVAL;
  if (src_dtype != MOE_F32 && src_dtype != MOE_BF16) return MOE_EINVAL;
  if ((int64_t)rows * cols >= ((int64_t)1 << 40)) return MOE_EUNSUPPORTED;
  if (block_rows == 128 && (rows + 127) / 128 > 65535) return MOE_EUNSUPPORTED;
  if (rows == 0 || cols == 0) return MOE_OK;
  if (!src || !codes || !scales) return MOE_EINVAL;
  if (!aligned(src, 16) || !aligned(codes, 8) || !aligned(scales, 4)) return MOE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (block_rows == 1) {
    PROF_BEGIN("quant_rows", st);
    if (src_dtype == MOE_BF16)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fp8_quant_rows<bf16_t>), dim3((rows + 3) / 4), dim3(256),
                         0, st, (const bf16_t*)src, rows, cols, codes, scales);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fp8_quant_rows<float>), dim3((rows + 3) / 4), dim3(256),
                         0, st, (const float*)src, rows, cols, codes, scales);
    PROF_END("quant_rows", st);
  } else {
    const dim3 g(cols / 128, (rows + 127) / 128);
    if (src_dtype == MOE_BF16)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fp8_quant_tiles<bf16_t>), g, dim3(256), 0, st,
                         (const bf16_t*)src, rows, cols, codes, scales);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(fp8_quant_tiles<float>), g, dim3(256), 0, st,
                         (const float*)src, rows, cols, codes, scales);
  }
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

namespace {

// The gather-fused BF16 expert products; with AB the first product also
// stores its pre-activations [A|B] for the backward.
moe_status ffn_gather_impl(const moe_cfg* cfg, const void* X, const int32_t* row_map,
                           const int32_t* offsets, const void* W13, const void* W2, void* Y,
                           void* AB, void* ws, size_t ws_bytes, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.act != MOE_BF16 || c.w != MOE_BF16) return MOE_EUNSUPPORTED;
  if (c.d_ff % 128 != 0 || c.d % 256 != 0) return MOE_EUNSUPPORTED;
  if (!offsets || !W13 || !W2) return MOE_EINVAL;
  if (c.T > 0 && (!X || !row_map || !Y)) return MOE_EINVAL;
  if (!aligned(X, 16) || !aligned(W13, 16) || !aligned(W2, 16) || !aligned(Y, 16) ||
      !aligned(offsets, 4) || !aligned(row_map, 4) || !aligned(AB, 16))
    return MOE_EINVAL;
  if (ws_bytes < ffn_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  if (c.T == 0) return MOE_OK;
  hipStream_t st = (hipStream_t)stream;
  FfnWs w = carve_ffn(c, ws, nullptr);
  const int N = c.T * c.k;
  hipLaunchKernelGGL(ffn_tiles, dim3(1), dim3(1024), 0, st, offsets, c.E, GBM, w.tile_start_big);
  const int mt_big = (N + GBM - 1) / GBM + c.E;
  {
    const int nt = c.d_ff / 128;
    const int G = (mt_big * nt + 7) / 8 * 8;
    PROF_BEGIN("gemm1_swiglu", st);
    if (AB)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_bf16_wide<EPI_SWIGLU_AB, true>), dim3(G),
                         dim3(64 * XW), 0, st, (const bf16_t*)X, row_map, c.T,
                         (const bf16_t*)W13, (bf16_t*)w.h, offsets, w.tile_start_big, c.E, N, c.d,
                         c.d_ff, c.d_ff, nt, G, (bf16_t*)AB);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_bf16_wide<EPI_SWIGLU, true>), dim3(G),
                         dim3(64 * XW), 0, st, (const bf16_t*)X, row_map, c.T,
                         (const bf16_t*)W13, (bf16_t*)w.h, offsets, w.tile_start_big, c.E, N, c.d,
                         c.d_ff, c.d_ff, nt, G, nullptr);
    PROF_END("gemm1_swiglu", st);
  }
  {
    const int nt = c.d / 256;
    const int G = (mt_big * nt + 7) / 8 * 8;
    PROF_BEGIN("gemm2", st);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_bf16_wide<EPI_PLAIN, false>), dim3(G), dim3(64 * XW),
                       0, st, (const bf16_t*)w.h, nullptr, 0, (const bf16_t*)W2, (bf16_t*)Y,
                       offsets, w.tile_start_big, c.E, N, c.d_ff, c.d_ff, c.d, nt, G, nullptr);
    PROF_END("gemm2", st);
  }
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

}  // namespace

extern "C" moe_status moe_expert_ffn_gather(const moe_cfg* cfg, const void* X,
                                            const int32_t* row_map, const int32_t* offsets,
                                            const void* W13, const void* W2, void* Y, void* ws,
                                            size_t ws_bytes, void* stream) {
  return ffn_gather_impl(cfg, X, row_map, offsets, W13, W2, Y, nullptr, ws, ws_bytes, stream);
}

extern "C" moe_status moe_expert_ffn_gather_save(const moe_cfg* cfg, const void* X,
                                                 const int32_t* row_map, const int32_t* offsets,
                                                 const void* W13, const void* W2, void* Y,
                                                 void* AB, void* ws, size_t ws_bytes,
                                                 void* stream) {
  if (cfg && cfg->T > 0 && !AB) return MOE_EINVAL;
  return ffn_gather_impl(cfg, X, row_map, offsets, W13, W2, Y, AB, ws, ws_bytes, stream);
}

extern "C" moe_status moe_expert_ffn_gather_fp8(const moe_cfg* cfg, const uint8_t* X_codes,
                                                const float* X_scale, const int32_t* row_map,
                                                const int32_t* offsets, const uint8_t* W13,
                                                const float* W13_scale, const uint8_t* W2,
                                                const float* W2_scale, void* Y, void* ws,
                                                size_t ws_bytes, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.act != MOE_BF16 || c.w != MOE_FP8E4M3) return MOE_EUNSUPPORTED;
  if (c.d_ff % 128 != 0 || c.d % 128 != 0) return MOE_EUNSUPPORTED;
  if (!offsets || !W13 || !W2 || !W13_scale || !W2_scale) return MOE_EINVAL;
  if (c.T > 0 && (!X_codes || !X_scale || !row_map || !Y)) return MOE_EINVAL;
  if (!aligned(X_codes, 16) || !aligned(X_scale, 4) || !aligned(W13, 16) || !aligned(W2, 16) ||
      !aligned(Y, 16) || !aligned(offsets, 4) || !aligned(row_map, 4) ||
      !aligned(W13_scale, 4) || !aligned(W2_scale, 4))
    return MOE_EINVAL;
  if (ws_bytes < ffn_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  if (c.T == 0) return MOE_OK;
  hipStream_t st = (hipStream_t)stream;
  FfnWs w = carve_ffn(c, ws, nullptr);
  launch_fp8_ffn(c, w, (const fp8_t*)X_codes, X_scale, row_map, offsets, (const fp8_t*)W13,
                 W13_scale, (const fp8_t*)W2, W2_scale, (bf16_t*)Y, st);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

extern "C" moe_status moe_quantize_mx(int rows, int cols, int fmt, int src_dtype, const void* src,
                                      uint8_t* codes, uint8_t* scales, void* stream) {
  const int hw = mx_format(fmt);
  if (hw < 0) return MOE_EINVAL;
  if (rows < 0 || cols < 0 || cols % 32 != 0) return MOE_EINVAL;
  if (src_dtype != MOE_F32 && src_dtype != MOE_BF16) return MOE_EINVAL;
  if ((int64_t)rows * cols >= ((int64_t)1 << 40)) return MOE_EUNSUPPORTED;
  if (rows == 0 || cols == 0) return MOE_OK;
  if (!src || !codes || !scales) return MOE_EINVAL;
  if (!aligned(src, 16) || !aligned(codes, 16) || !aligned(scales, 4)) return MOE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const size_t nblk = (size_t)rows * (cols / 32);
  const dim3 g((unsigned)((nblk + 255) / 256));
  PROF_BEGIN("quant_mx", st);
#define MX_Q(F)                                                                               \
  if (src_dtype == MOE_BF16)                                                                  \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(mx_quant_rows<F, bf16_t>), g, dim3(256), 0, st,        \
                       (const bf16_t*)src, rows, cols, codes, scales);                        \
  else                                                                                        \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(mx_quant_rows<F, float>), g, dim3(256), 0, st,         \
                       (const float*)src, rows, cols, codes, scales);
  if (hw == 0) { MX_Q(0) }
  else if (hw == 2) { MX_Q(2) }
  else { MX_Q(4) }
#undef MX_Q
  PROF_END("quant_mx", st);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

extern "C" moe_status moe_expert_ffn_mx(const moe_cfg* cfg, const uint8_t* X_codes,
                                        const uint8_t* X_scale, const int32_t* row_map,
                                        const int32_t* offsets, const uint8_t* W13,
                                        const uint8_t* W13_scale, const uint8_t* W2,
                                        const uint8_t* W2_scale, void* Y, void* ws,
                                        size_t ws_bytes, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  const int hw = mx_format(c.w);
  if (c.act != MOE_BF16 || hw < 0) return MOE_EUNSUPPORTED;
  if (c.d % 256 != 0 || c.d_ff % 128 != 0) return MOE_EUNSUPPORTED;
  if (!offsets || !W13 || !W2 || !W13_scale || !W2_scale) return MOE_EINVAL;
  if (c.T > 0 && (!X_codes || !X_scale || !row_map || !Y)) return MOE_EINVAL;
  if (!aligned(X_codes, 16) || !aligned(X_scale, 4) || !aligned(W13, 16) || !aligned(W2, 16) ||
      !aligned(W13_scale, 4) || !aligned(W2_scale, 4) || !aligned(Y, 16) ||
      !aligned(offsets, 4) || !aligned(row_map, 4))
    return MOE_EINVAL;
  if (ws_bytes < ffn_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  if (c.T == 0) return MOE_OK;
  hipStream_t st = (hipStream_t)stream;
  FfnWs w = carve_ffn(c, ws, nullptr);
  const int N = c.T * c.k;
  hipLaunchKernelGGL(ffn_tiles, dim3(1), dim3(1024), 0, st, offsets, c.E, GBM, w.tile_start_big);
  const int mt_big = (N + GBM - 1) / GBM + c.E;
  const int nt1 = c.d_ff / 128, G1 = (mt_big * nt1 + 7) / 8 * 8;
  const int nt2 = c.d / 256, G2 = (mt_big * nt2 + 7) / 8 * 8;
#define MX_FFN(F)                                                                              \
  {                                                                                            \
    PROF_BEGIN("gemm1_swiglu", st);                                                            \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_mx_wide<F, EPI_SWIGLU, true>), dim3(G1),           \
                       dim3(64 * XW), 0, st, X_codes, X_scale, row_map, c.T, W13, W13_scale,   \
                       w.h, w.hx, offsets, w.tile_start_big, c.E, N, c.d, c.d_ff, c.d_ff, nt1, \
                       G1);                                                                    \
    PROF_END("gemm1_swiglu", st);                                                              \
    PROF_BEGIN("gemm2", st);                                                                   \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(gemm_mx_wide<F, EPI_PLAIN, false>), dim3(G2),           \
                       dim3(64 * XW), 0, st, (const uint8_t*)w.h, (const uint8_t*)w.hx,        \
                       nullptr, 0, W2, W2_scale, Y, nullptr, offsets, w.tile_start_big, c.E, N, \
                       c.d_ff, c.d_ff, c.d, nt2, G2);                                          \
    PROF_END("gemm2", st);                                                                     \
  }
  if (hw == 0) MX_FFN(0)
  else if (hw == 2) MX_FFN(2)
  else MX_FFN(4)
#undef MX_FFN
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

// ---------------------------------------------------- counter calibration
namespace {
__global__ __launch_bounds__(256) void lds_copy_kernel(const u32x4* __restrict__ src,
                                                       u32x4* __restrict__ dst, size_t n16) {
  typedef __attribute__((address_space(3))) void lds_void;
  __shared__ __attribute__((aligned(1024))) u32x4 buf[256];
  const int tid = threadIdx.x, wv = tid >> 6;
  for (size_t off = (size_t)blockIdx.x * 256; off < n16; off += (size_t)gridDim.x * 256) {
    if (off + 256 <= n16) {
      // each wavefront deposits its 64 x 16 bytes contiguously
      __builtin_amdgcn_global_load_lds(src + off + tid, (lds_void*)(buf + wv * 64), 16, 0, 0);
      WAIT_VM_LGKM0(0);
      __syncthreads();
      dst[off + tid] = buf[tid];
      __syncthreads();
    } else if (off + tid < n16) {
      dst[off + tid] = src[off + tid];
    }
  }
}
}  // namespace

extern "C" moe_status moe_prof_lds_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (bytes % 16 != 0 || !aligned(src, 16) || !aligned(dst, 16)) return MOE_EINVAL;
  if (bytes == 0) return MOE_OK;
  if (!src || !dst) return MOE_EINVAL;
  const size_t n16 = bytes / 16;
  const size_t blocks = (n16 + 255) / 256;
  const unsigned g = (unsigned)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(lds_copy_kernel, dim3(g), dim3(256), 0, (hipStream_t)stream,
                     (const u32x4*)src, (u32x4*)dst, n16);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}
