// Matrix-core GEMM kernels for gfx950 (FP64 and BF16 with FP32 accumulation).
//
// One work-group of 256 lanes (4 wave64s in a 2 x 2 arrangement) computes a
// BM x BN tile of C.  K is walked in BK slices staged through LDS with two
// buffers: the next slice is fetched into registers while the matrix cores
// work on the current one, so each slice costs a single barrier.
//
// LDS layouts are chosen for the fragment reads of each instruction:
//  * v_mfma_f64_16x16x4f64: lane l needs A(l%16, l/16) and B(l/16, l%16), one
//    double each, so tiles are kept k-major (As[k][m], Bs[k][n]); its result
//    element (i, j) is register i/4 of lane j + 16 (i%4);
//  * v_mfma_f32_16x16x32_bf16: lane l needs 8 consecutive k of row l%16; a
//    k-contiguous operand is kept [row][k] with XOR-swizzled 16-byte chunks
//    (see BfTile), a row-contiguous one [k][row] as loaded and read with a
//    transposing LDS load; its result element (i, j) is register i%4 of lane
//    j + 16 (i/4).
// Global reads stay coalesced in both cases.
// Work-group ids are remapped so that each XCD owns a contiguous range of
// tiles, and inside a batch the tile dimension with fewer tiles runs fastest,
// so the larger operand is streamed from HBM about once.
#include "gemm.h"

#include "fp8.h"

#include <algorithm>
#include <type_traits>
#include <stdexcept>

namespace cpppl {

namespace {

struct KArgs {
  int64_t M, N, K, batch;
  const void* A;
  int64_t sam, sak, sab;
  const void* B;
  int64_t sbk, sbn, sbb;
  void* C;
  int64_t scm, scb;
  double alpha, beta;
  int splits;
  int64_t kchunk;
  void* partial;
  int64_t tiles_m, tiles_n;
  int vec_ok;    // 16-byte operand loads allowed (8-byte for e4m3 B)
  int cvec_ok;   // 16-byte result stores allowed
  const float* bscale;  // e4m3 B: scale per column (mode 1) or per k (mode 2)
  int bscale_mode;
};

struct Coords {
  int64_t b, tm, tn;
  int split;
};

__device__ __forceinline__ Coords tile_coords(int64_t lid, const KArgs& a) {
  const int64_t tiles = a.tiles_m * a.tiles_n;
  const int64_t t = lid % tiles;
  const int64_t bs = lid / tiles;
  Coords c;
  c.split = (int)(bs % a.splits);
  c.b = bs / a.splits;
  if (a.tiles_m <= a.tiles_n) {
    c.tm = t % a.tiles_m;
    c.tn = t / a.tiles_m;
  } else {
    c.tn = t % a.tiles_n;
    c.tm = t / a.tiles_n;
  }
  return c;
}

// 32-bit form of xcd_remap followed by tile_coords, for launches whose tile
// count is below 2^31 (the BF16 launcher refuses larger grids).
__device__ __forceinline__ Coords tile_coords32(uint32_t bid, uint32_t nblocks, const KArgs& a) {
  uint32_t lid = bid;
  if (nblocks >= 8) {
    const uint32_t per = nblocks / 8, rem = nblocks % 8, xcd = bid % 8;
    lid = xcd * per + (xcd < rem ? xcd : rem) + bid / 8;
  }
  const uint32_t tmn = (uint32_t)a.tiles_m, tnn = (uint32_t)a.tiles_n;
  const uint32_t tiles = tmn * tnn;
  const uint32_t t = lid % tiles, bs = lid / tiles;
  const uint32_t sp = (uint32_t)a.splits;
  Coords c;
  c.split = (int)(bs % sp);
  c.b = bs / sp;
  if (tmn <= tnn) {
    c.tm = t % tmn;
    c.tn = t / tmn;
  } else {
    c.tn = t % tnn;
    c.tm = t / tnn;
  }
  return c;
}

template <typename OutT>
__device__ __forceinline__ void store_out(const KArgs& a, const Coords& tc, int64_t gm, int64_t gn,
                                          double v) {
  if (a.splits > 1) {
    const int64_t off = ((int64_t)tc.split * a.batch + tc.b) * a.M * a.N + gm * a.N + gn;
    if constexpr (sizeof(OutT) == 8) ((double*)a.partial)[off] = v;
    else ((float*)a.partial)[off] = (float)v;
    return;
  }
  OutT* c = (OutT*)a.C + tc.b * a.scb + gm * a.scm + gn;
  double r = a.alpha * v;
  if (a.beta != 0.0) r += a.beta * Conv<OutT>::to_f64(*c);
  *c = Conv<OutT>::from_f64(r);
}

// ------------------------------------------------------------------ FP64 ----
template <int BM, int BN, bool AK, bool BKC>
__global__ __launch_bounds__(256, BM > 64 ? 2 : 1) void gemm_f64_kernel(const KArgs a) {
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  __shared__ double As[2][BK][BM + 1];
  __shared__ double Bs[2][BK][BN + 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const Coords tc = tile_coords(xcd_remap(blockIdx.x, gridDim.x), a);
  const int64_t m0 = tc.tm * BM, n0 = tc.tn * BN;
  const int64_t kbeg = (int64_t)tc.split * a.kchunk;
  const int64_t kend = min(a.K, kbeg + a.kchunk);
  const double* A = (const double*)a.A + tc.b * a.sab;
  const double* B = (const double*)a.B + tc.b * a.sbb;

  double ra[EA], rb[EB];
  d4_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

#define F64_GLOAD(k0)                                                                        \
  {                                                                                          \
    _Pragma("unroll") for (int e = 0; e < EA; ++e) {                                         \
      const int idx = tid + e * 256;                                                         \
      const int mm = AK ? idx / BK : idx % BM;                                               \
      const int kk = AK ? idx % BK : idx / BM;                                               \
      const int64_t gm = m0 + mm, gk = (k0) + kk;                                            \
      ra[e] = (gm < a.M && gk < kend) ? A[AK ? (gm * a.sam + gk) : (gm + gk * a.sak)] : 0.0; \
    }                                                                                        \
    _Pragma("unroll") for (int e = 0; e < EB; ++e) {                                         \
      const int idx = tid + e * 256;                                                         \
      const int nn = BKC ? idx / BK : idx % BN;                                              \
      const int kk = BKC ? idx % BK : idx / BN;                                              \
      const int64_t gn = n0 + nn, gk = (k0) + kk;                                            \
      rb[e] = (gn < a.N && gk < kend) ? B[BKC ? (gn * a.sbn + gk) : (gn + gk * a.sbk)] : 0.0; \
    }                                                                                        \
  }
#define F64_SSTORE(buf)                                  \
  {                                                      \
    _Pragma("unroll") for (int e = 0; e < EA; ++e) {     \
      const int idx = tid + e * 256;                     \
      const int mm = AK ? idx / BK : idx % BM;           \
      const int kk = AK ? idx % BK : idx / BM;           \
      As[buf][kk][mm] = ra[e];                           \
    }                                                    \
    _Pragma("unroll") for (int e = 0; e < EB; ++e) {     \
      const int idx = tid + e * 256;                     \
      const int nn = BKC ? idx / BK : idx % BN;          \
      const int kk = BKC ? idx % BK : idx / BN;          \
      Bs[buf][kk][nn] = rb[e];                           \
    }                                                    \
  }

  const int64_t nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    F64_GLOAD(kbeg);
    F64_SSTORE(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nk) F64_GLOAD(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = As[cur][ks + (lane >> 4)][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = Bs[cur][ks + (lane >> 4)][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) F64_SSTORE(cur ^ 1);
    __syncthreads();
  }
#undef F64_GLOAD
#undef F64_SSTORE

  // v_mfma_f64_16x16x4f64 result layout: element (i, j) of the 16 x 16 tile is
  // register i / 4 of lane j + 16 * (i % 4).
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * WM + i * 16 + 4 * r + (lane >> 4);
        const int64_t gn = n0 + wn * WN + j * 16 + (lane & 15);
        if (gm < a.M && gn < a.N) store_out<double>(a, tc, gm, gn, acc[i][j][r]);
      }
}

// ------------------------------------------------------------------ BF16 ----
// K slice: 32 for short K (4 work-groups per CU hide more latency), 64 for
// long K per split (fewer barriers per flop).
constexpr int BBK_SHORT = 32, BBK_LONG = 64;
constexpr int64_t BBK_LONG_MIN_K = 2048;
// Chained launches (two tiles per work-group): products of 2048 to 4096
// tiles of 128 x 128 whose K per split is at most 512.
constexpr int64_t BF16_CHAIN_MIN_TILES = 2048, BF16_CHAIN_MAX_TILES = 4096,
                  BF16_CHAIN_MAX_K = 512;

// 16 aligned bytes as one vector load (a plain uint4 copy can be lowered to a
// memcpy through private memory).
__device__ __forceinline__ uint4 load16(const bf16_t* p) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = *(const u32x4*)p;
  return make_uint4(v[0], v[1], v[2], v[3]);
}

// 8 bf16 at p[0], p[step], ... with the elements at index >= count set to 0.
__device__ __forceinline__ uint4 gather8(const bf16_t* p, int64_t step, int64_t count) {
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = (2 * q < count) ? (uint32_t)p[(2 * q) * step] : 0u;
    const uint32_t hi = (2 * q + 1 < count) ? (uint32_t)p[(2 * q + 1) * step] : 0u;
    w[q] = lo | (hi << 16);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

typedef short s4_t __attribute__((ext_vector_type(4)));

// ds_read_b64_tr_b16: within each group of 16 lanes, lane i receives element
// i % 4 of the 8 bytes addressed by lane 4 c + i / 4 as its component c.
__device__ __forceinline__ s4_t lds_read_tr(const bf16_t* p) {
  typedef __attribute__((address_space(3))) s4_t lds_s4;
  return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s4*)(__attribute__((address_space(3))) void*)p);
}

// One operand tile (ROWS x BBK) of a BF16 GEMM: global -> registers -> LDS.
// KC: the operand's unit stride is along k; the tile is kept [row][k] with
// unpadded rows and a fragment is one 16-byte read.  The 16-byte chunk index is
// XOR-ed with (row >> 1) & 3 (BBK = 32, 64-byte rows) or row & 7 (BBK = 64,
// 128-byte rows): measured on gfx950 with the LDS bank-conflict counter, this
// makes both the tile stores (4 or 8 lanes per row) and the fragment reads
// (16 rows, one chunk) conflict-free, where a swizzle by row bits 2-3, plain
// rows or 144-byte padded rows leave the fragment reads two-way conflicted.
// Otherwise the unit stride is along the row index; the tile is kept [k][row]
// (16-byte stores straight from the coalesced loads, rows padded to 288 bytes so
// the 16 rows read by one transposing instruction fall on disjoint bank groups)
// and a fragment is two transposing reads.
template <int ROWS, bool KC, int BBK, int NT = 256>
struct BfTile {
  static constexpr int BLDK = BBK;                      // row pitch of the [row][k] layout
  static_assert(ROWS * BBK % (8 * NT) == 0, "tile chunks must divide evenly over the lanes");
  static constexpr int C = ROWS * BBK / 8 / NT;
  static constexpr int LDT = ROWS + 16;                 // row pitch of the [k][row] layout
  static constexpr int SIZE = KC ? ROWS * BLDK : BBK * LDT;  // bf16 elements per buffer
  // element offset of (row, kk) in the [row][k] layout, kk a multiple of 8
  __device__ __forceinline__ static int kc_off(int row, int kk) {
    const int swz = BBK == 32 ? (row >> 1) & 3 : row & 7;
    return row * BLDK + (((kk >> 3) ^ swz) << 3);
  }
  // FAST: every 16-byte chunk of the slice lies inside K (K a multiple of the
  // slice) and is aligned; rows past the end are clamped to the last row
  // (the last aligned group of 8 for a row-contiguous operand, whose row count
  // is then a multiple of 8): they only feed results that are not stored.
  template <bool FAST = false>
  __device__ __forceinline__ static void load(uint4 (&r)[C], const bf16_t* X, int64_t s_row,
                                              int64_t s_k, int64_t row0, int64_t nrows, int64_t k0,
                                              int64_t kend, bool vec, int tid) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const int c = tid + e * NT;
      if constexpr (FAST && KC) {
        const int row = c / (BBK / 8), kk = (c % (BBK / 8)) * 8;
        const int64_t g = min(row0 + row, nrows - 1);
        r[e] = load16(X + g * s_row + k0 + kk);
      } else if constexpr (FAST) {
        const int kk = c / (ROWS / 8), row = (c % (ROWS / 8)) * 8;
        const int64_t g = min(row0 + row, nrows - 8);
        r[e] = load16(X + (k0 + kk) * s_k + g);
      } else if (KC) {
        const int row = c / (BBK / 8), kk = (c % (BBK / 8)) * 8;
        const int64_t g = row0 + row, gk = k0 + kk;
        const bf16_t* p = X + g * s_row + gk;
        if (vec && g < nrows && gk + 8 <= kend) r[e] = *(const uint4*)p;
        else r[e] = gather8(p, 1, g < nrows ? kend - gk : 0);
      } else {
        const int kk = c / (ROWS / 8), row = (c % (ROWS / 8)) * 8;
        const int64_t g = row0 + row, gk = k0 + kk;
        const bf16_t* p = X + gk * s_k + g;
        if (vec && gk < kend && g + 8 <= nrows) r[e] = *(const uint4*)p;
        else r[e] = gather8(p, 1, gk < kend ? nrows - g : 0);
      }
    }
  }
  __device__ __forceinline__ static void store(const uint4 (&r)[C], bf16_t* S, int tid) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const int c = tid + e * NT;
      if (KC) {
        const int row = c / (BBK / 8), kk = (c % (BBK / 8)) * 8;
        *(uint4*)&S[kc_off(row, kk)] = r[e];
      } else {
        const int kk = c / (ROWS / 8), row = (c % (ROWS / 8)) * 8;
        *(uint4*)&S[kk * LDT + row] = r[e];
      }
    }
  }
  // Matrix-core fragment of rows row0 .. row0 + 15, k = ks .. ks + 31: lane l
  // gets row row0 + l % 16, k = ks + 8 (l / 16) .. + 7.
  __device__ __forceinline__ static bf16x8_t frag(const bf16_t* S, int row0, int ks, int lane) {
    if (KC) {
      return *(const bf16x8_t*)&S[kc_off(row0 + (lane & 15), ks + 8 * (lane >> 4))];
    } else {
      const int s = lane & 15;
      const bf16_t* p = &S[(ks + 8 * (lane >> 4) + (s >> 2)) * LDT + row0 + 4 * (s & 3)];
      const s4_t lo = lds_read_tr(p);
      const s4_t hi = lds_read_tr(p + 4 * LDT);
      typedef short s8_t __attribute__((ext_vector_type(8)));
      const s8_t v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      return __builtin_bit_cast(bf16x8_t, v);
    }
  }
};

// A k-contiguous B tile stored as e4m3 codes: each lane keeps its chunks of 8
// codes (8 bytes) and their scale in registers while the matrix cores work on
// the previous slice, then writes them to LDS as bfloat16 in the layout of
// BfTile<ROWS, true, BBK>, so the fragment reads are those of the BF16 kernel.
template <int ROWS, int BBK>
struct F8Tile {
  using L = BfTile<ROWS, true, BBK>;
  static constexpr int C = L::C;
  struct Regs {
    uint2 q[C];
    float s[C];
  };
  // scales that do not change along k (mode 0: 1, mode 1: per row)
  __device__ __forceinline__ static void init_scales(Regs& r, const KArgs& a, int64_t row0,
                                                     int64_t nrows, int tid) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const int64_t g = row0 + (tid + e * 256) / (BBK / 8);
      r.s[e] = (a.bscale_mode == 1 && g < nrows) ? a.bscale[g] : 1.0f;
    }
  }
  // FAST as for BfTile::load: whole aligned chunks, rows clamped.
  template <bool FAST = false>
  __device__ __forceinline__ static void load(Regs& r, const uint8_t* X, int64_t s_row, int64_t row0,
                                              int64_t nrows, int64_t k0, int64_t kend, bool vec,
                                              const KArgs& a, int tid) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const int c = tid + e * 256;
      const int row = c / (BBK / 8), kk = (c % (BBK / 8)) * 8;
      const int64_t g = FAST ? min(row0 + row, nrows - 1) : row0 + row, gk = k0 + kk;
      const uint8_t* p = X + g * s_row + gk;
      if constexpr (FAST) {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 v = *(const u32x2*)p;
        r.q[e] = make_uint2(v[0], v[1]);
      } else if (vec && g < nrows && gk + 8 <= kend) {
        r.q[e] = *(const uint2*)p;
      } else {
        const int64_t cnt = g < nrows ? kend - gk : 0;
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < cnt) w[q >> 2] |= (uint32_t)p[q] << (8 * (q & 3));
        r.q[e] = make_uint2(w[0], w[1]);
      }
      if (a.bscale_mode == 2) r.s[e] = (FAST || gk < kend) ? a.bscale[gk] : 1.0f;
    }
  }
  __device__ __forceinline__ static void store(const Regs& r, bf16_t* S, int tid) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const int c = tid + e * 256;
      const int row = c / (BBK / 8), kk = (c % (BBK / 8)) * 8;
      *(uint4*)&S[L::kc_off(row, kk)] = e4m3x8_to_bf16(r.q[e], r.s[e]);
    }
  }
};

template <typename OutT>
__device__ __forceinline__ OutT to_out(float v);
template <> __device__ __forceinline__ float to_out<float>(float v) { return v; }
template <> __device__ __forceinline__ bf16_t to_out<bf16_t>(float v) { return f32_to_bf16(v); }
template <> __device__ __forceinline__ double to_out<double>(float v) { return (double)v; }

// Waves per SIMD (work-groups per CU for 128 x 128 tiles): 4 where the
// registers fit in 128 (two k-contiguous operands, or two row-contiguous ones
// with unchecked loads, 2- or 4-byte results), else 3; 2 for K slices of 64.
template <bool AK, bool BKC, bool B8, bool FAST, typename OutT>
constexpr bool four_waves() {
  return ((AK && BKC) || (FAST && !AK && !BKC)) && !B8 && sizeof(OutT) <= 4;
}
// WGM wave rows by 2 wave columns: 4 waves (128 x 128 tiles) or 8 waves
// (256 x 128 tiles, two per CU: each operand element staged in LDS then feeds
// 256 or 128 products instead of 128, a quarter less LDS writing and L2
// reading per flop at the same 64 x 64 tile per wave).
template <int BM, int BN, int BBK, bool AK, bool BKC, typename OutT, bool B8 = false, int WGM = 2,
          bool FAST = false>
__global__ __launch_bounds__(128 * WGM, WGM == 4 ? 4 : (BBK == BBK_LONG ? 2 : (four_waves<AK, BKC, B8, FAST, OutT>() ? 4 : 3)))
void gemm_bf16_kernel(const KArgs a) {
  static_assert(!B8 || BKC, "an e4m3 B operand must be k-contiguous");
  static_assert(WGM == 2 || (WGM == 4 && BBK == BBK_SHORT && AK && BKC && !B8),
                "8-wave tiles: k-contiguous BF16 operands, short slices");
  constexpr int NT = 128 * WGM;
  constexpr int WM = BM / WGM, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  using TA = BfTile<BM, AK, BBK, NT>;
  using TB = BfTile<BN, BKC, BBK, NT>;
  constexpr int AS = TA::SIZE, BS = TB::SIZE;  // bf16 elements per buffer
  // staged epilogue: 2-byte results in passes of 128 rows (two wave rows),
  // 4-byte results (FP32 output or split-K partials) in passes of one wave row
  constexpr bool STAGE = sizeof(OutT) <= 4;
  constexpr int LDC2 = BN + 8, LDC4 = BN + 4;
  constexpr int SMEM_AB = 2 * (AS + BS) * 2;
  constexpr int SMEM_C2 = 2 * WM * LDC2 * 2, SMEM_C4 = WM * LDC4 * 4;
  constexpr int SMEM_C = SMEM_C2 > SMEM_C4 ? SMEM_C2 : SMEM_C4;
  constexpr int SMEM = SMEM_AB > SMEM_C ? SMEM_AB : SMEM_C;
  __shared__ __attribute__((aligned(16))) char smem[SMEM];
  bf16_t* As = (bf16_t*)smem;             // [2][AS]
  bf16_t* Bs = (bf16_t*)smem + 2 * AS;    // [2][BS]

  const int tid0 = threadIdx.x;
  const bool vec = a.vec_ok != 0;
  const int64_t sa_row = AK ? a.sam : 1, sa_k = AK ? 1 : a.sak;
  const int64_t sb_row = BKC ? a.sbn : 1, sb_k = BKC ? 1 : a.sbk;

  // A work-group computes the tiles blockIdx.x, blockIdx.x + gridDim.x, ...
  // of the XCD-remapped order (one tile when the grid covers them all).
  const uint32_t ntile = (uint32_t)(a.tiles_m * a.tiles_n * a.batch * a.splits);
  using T8 = F8Tile<BN, BBK>;
  uint4 ra[TA::C], rb[B8 ? 1 : TB::C];
  typename T8::Regs r8;
  // A second register stage keeps the global loads of slice k + 2 in flight
  // while slice k is multiplied: for long K slices (two work-groups per CU),
  // and on the unchecked path where it costs no occupancy (256-row tiles, and
  // 128 x 128 tiles already at three waves per SIMD).  Measured on MI355X, it
  // costs more than it gains where it would take a fourth wave away.
  constexpr bool DEEP =
      !B8 && (BBK == BBK_LONG || (FAST && (WGM == 4 || !four_waves<AK, BKC, B8, FAST, OutT>())));
  // Chained tiles (unchecked single-stage path only): the loads of the next
  // tile's first slice are issued before this tile's epilogue, so they are in
  // flight while its results are stored.
  constexpr bool CHAIN = FAST && WGM == 2 && !DEEP && !B8;
  bool primed = false;  // ra, rb hold the first slice of the current tile
  Coords tc = tile_coords32(blockIdx.x, ntile, a);
  for (uint32_t vt = blockIdx.x; vt < ntile; vt += gridDim.x) {
    // lane-dependent addresses are recomputed per tile rather than held in
    // registers across the tile loop
    int tid = tid0;
    if constexpr (CHAIN) asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const uint32_t vnext = vt + gridDim.x;
    const bool more = CHAIN && vnext < ntile;
    const Coords tn = more ? tile_coords32(vnext, ntile, a) : tc;
    const int64_t m0 = tc.tm * BM, n0 = tc.tn * BN;
    const int64_t kbeg = (int64_t)tc.split * a.kchunk;
    const int64_t kend = min(a.K, kbeg + a.kchunk);
    const bf16_t* A = (const bf16_t*)a.A + tc.b * a.sab;
    const bf16_t* B = (const bf16_t*)a.B + tc.b * a.sbb;

    if constexpr (B8) T8::init_scales(r8, a, n0, a.N, tid);
    f4_t acc[TM][TN];
  #pragma unroll
    for (int i = 0; i < TM; ++i)
  #pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

    const int64_t nk = kend > kbeg ? (kend - kbeg + BBK - 1) / BBK : 0;
    if (nk > 0) {
      if (!primed) {
        TA::template load<FAST>(ra, A, sa_row, sa_k, m0, a.M, kbeg, kend, vec, tid);
        if constexpr (B8)
          T8::template load<FAST>(r8, (const uint8_t*)a.B + tc.b * a.sbb, a.sbn, n0, a.N, kbeg, kend,
                                  vec, a, tid);
        else TB::template load<FAST>(rb, B, sb_row, sb_k, n0, a.N, kbeg, kend, vec, tid);
      }
      TA::store(ra, As, tid);
      if constexpr (B8) T8::store(r8, Bs, tid);
      else TB::store(rb, Bs, tid);
    }
    primed = false;
    auto mma = [&](const bf16_t* Ac, const bf16_t* Bc) {
  #pragma unroll
      for (int ks = 0; ks < BBK; ks += 32) {
        bf16x8_t af[TM], bfr[TN];
  #pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = TA::frag(Ac, wm * WM + i * 16, ks, lane);
  #pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = TB::frag(Bc, wn * WN + j * 16, ks, lane);
  #pragma unroll
        for (int i = 0; i < TM; ++i)
  #pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
      }
    };
    if constexpr (DEEP) {
      uint4 ra2[TA::C], rb2[TB::C];
      // With unchecked loads the slice index is clamped instead of the loads
      // being skipped past the end (a repeated last slice is never stored):
      // loads issued on every path let the compiler wait for one stage only.
      if (FAST || nk > 1) {
        const int64_t k1 = kbeg + (FAST ? min((int64_t)1, nk - 1) : 1) * BBK;
        TA::template load<FAST>(ra2, A, sa_row, sa_k, m0, a.M, k1, kend, vec, tid);
        TB::template load<FAST>(rb2, B, sb_row, sb_k, n0, a.N, k1, kend, vec, tid);
      }
      __syncthreads();
      // slice kt sits in LDS buffer kt % 2; register stage kt % 2 is free and
      // receives slice kt + 2; stage (kt + 1) % 2 holds slice kt + 1
      auto step = [&](int64_t kt, uint4 (&la)[TA::C], uint4 (&lb)[TB::C], uint4 (&sa)[TA::C],
                      uint4 (&sb)[TB::C]) {
        const int cur = (int)(kt & 1);
        if (FAST || kt + 2 < nk) {
          const int64_t k2 = kbeg + (FAST ? min(kt + 2, nk - 1) : kt + 2) * BBK;
          TA::template load<FAST>(la, A, sa_row, sa_k, m0, a.M, k2, kend, vec, tid);
          TB::template load<FAST>(lb, B, sb_row, sb_k, n0, a.N, k2, kend, vec, tid);
        }
        mma(As + cur * AS, Bs + cur * BS);
        if (kt + 1 < nk) {
          TA::store(sa, As + (cur ^ 1) * AS, tid);
          TB::store(sb, Bs + (cur ^ 1) * BS, tid);
        }
        __syncthreads();
      };
      // Both steps run on every trip, so the loads in flight at the top of a
      // trip are always those into the second stage: the compiler then does not
      // wait for them before issuing the first stage's loads (a loop that could
      // come back after one step made it wait for every load in flight).
      int64_t kt = 0;
      for (; kt + 1 < nk; kt += 2) {
        step(kt, ra, rb, ra2, rb2);
        step(kt + 1, ra2, rb2, ra, rb);
      }
      if (kt < nk) step(kt, ra, rb, ra2, rb2);
    } else {
      __syncthreads();
      // the next tile's first slice, loaded after this tile's last one and
      // before its epilogue
      const int64_t nkbeg = (int64_t)tn.split * a.kchunk;
      const int64_t nkend = min(a.K, nkbeg + a.kchunk);
      const bool chain = CHAIN && more && nkend > nkbeg;
      for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const bf16_t* Ac = As + cur * AS;
        const bf16_t* Bc = Bs + cur * BS;
        if (kt + 1 < nk) {
          const int64_t k1 = kbeg + (kt + 1) * BBK;
          TA::template load<FAST>(ra, A, sa_row, sa_k, m0, a.M, k1, kend, vec, tid);
          if constexpr (B8)
            T8::template load<FAST>(r8, (const uint8_t*)a.B + tc.b * a.sbb, a.sbn, n0, a.N, k1, kend,
                                    vec, a, tid);
          else TB::template load<FAST>(rb, B, sb_row, sb_k, n0, a.N, k1, kend, vec, tid);
        }
        mma(Ac, Bc);
        if (kt + 1 < nk) {
          TA::store(ra, As + (cur ^ 1) * AS, tid);
          if constexpr (B8) T8::store(r8, Bs + (cur ^ 1) * BS, tid);
          else TB::store(rb, Bs + (cur ^ 1) * BS, tid);
        }
        __syncthreads();
      }
      if constexpr (CHAIN) {
        if (chain) {
          TA::template load<FAST>(ra, (const bf16_t*)a.A + tn.b * a.sab, sa_row, sa_k, tn.tm * BM, a.M,
                                  nkbeg, nkend, vec, tid);
          TB::template load<FAST>(rb, (const bf16_t*)a.B + tn.b * a.sbb, sb_row, sb_k, tn.tn * BN, a.N,
                                  nkbeg, nkend, vec, tid);
          primed = true;
        }
      }
    }

    // The products are formed as C^T = B^T A^T (B fragment first): element (m, n)
    // of a 16 x 16 block is register n % 4 of lane m + 16 (n / 4), so each lane
    // holds four consecutive columns of one row.
    if constexpr (STAGE) {
      // Stage the tile through LDS (the K-loop buffers are free after the last
      // barrier) and write whole 16-byte row chunks.
      const bool part = a.splits > 1;
      const int lr = lane & 15, lc = 4 * (lane >> 4);
      if (!part && sizeof(OutT) == 2) {
        bf16_t* Cs = (bf16_t*)smem;
        const float alpha = (float)a.alpha;
        constexpr int EPC = 8, CPR = BN / EPC, PROWS = 2 * WM;
        bf16_t* dst = (bf16_t*)a.C + tc.b * a.scb;
  #pragma unroll
        for (int pass = 0; pass < WGM / 2; ++pass) {
          if (pass > 0) __syncthreads();
          if ((wm >> 1) == pass) {
  #pragma unroll
            for (int i = 0; i < TM; ++i)
  #pragma unroll
              for (int j = 0; j < TN; ++j) {
                const int lm = (wm & 1) * WM + i * 16 + lr;
                const int ln = wn * WN + j * 16 + lc;
                // The hardware conversion (one instruction per pair) took Y, Z
                // and G 2-8 % faster alone at o = 32, v = 256, X = 768, R = 1024
                // (the sweep +1 %); in the 8-wave tile it pushed the kernel past
                // 128 registers into scratch (tau 9 % slower), so that tile keeps
                // the software rounding (the same result for every finite value).
                uint32_t w0, w1;
                if constexpr (WGM == 4) {
                  w0 = (uint32_t)f32_to_bf16(alpha * acc[i][j][0]) |
                       ((uint32_t)f32_to_bf16(alpha * acc[i][j][1]) << 16);
                  w1 = (uint32_t)f32_to_bf16(alpha * acc[i][j][2]) |
                       ((uint32_t)f32_to_bf16(alpha * acc[i][j][3]) << 16);
                } else {
                  w0 = pack_bf16x2(alpha * acc[i][j][0], alpha * acc[i][j][1]);
                  w1 = pack_bf16x2(alpha * acc[i][j][2], alpha * acc[i][j][3]);
                }
                *(uint2*)&Cs[lm * LDC2 + ln] = make_uint2(w0, w1);
              }
          }
          __syncthreads();
          for (int c = tid; c < PROWS * CPR; c += NT) {
            const int row = c / CPR, col = (c % CPR) * EPC;
            const int64_t gm = m0 + pass * PROWS + row, gn = n0 + col;
            if (gm >= a.M) continue;
            if (a.cvec_ok && gn + EPC <= a.N) {
              // Non-temporal: BF16 products (Y, Z, G, tau) stream to HBM and are
              // read back only by a later product.  Measured on MI355X at o = 32,
              // v = 256, X = 768, R = 1024: Y alone 0.248 -> 0.209 ms, the ALS
              // sweep +2 %.  (FP32 split-K partials, read back at once by the
              // reduction, keep ordinary stores: no gain measured there.)
              typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
              const u32x4 v = *(const u32x4*)(Cs + row * LDC2 + col);
              __builtin_nontemporal_store(v, (u32x4*)(dst + gm * a.scm + gn));
            } else {
              for (int q = 0; q < EPC; ++q)
                if (gn + q < a.N) dst[gm * a.scm + gn + q] = Cs[row * LDC2 + col + q];
            }
          }
        }
      } else {
        // FP32 results: split-K partials (row stride N, alpha applied later) or C
        float* Cs = (float*)smem;
        const float alpha = part ? 1.0f : (float)a.alpha;
        float* dst = part ? (float*)a.partial + ((int64_t)tc.split * a.batch + tc.b) * a.M * a.N
                          : (float*)a.C + tc.b * a.scb;
        const int64_t ldd = part ? a.N : a.scm;
        constexpr int EPC = 4, CPR = BN / EPC;
  #pragma unroll
        for (int pass = 0; pass < WGM; ++pass) {
          if (wm == pass) {
  #pragma unroll
            for (int i = 0; i < TM; ++i)
  #pragma unroll
              for (int j = 0; j < TN; ++j) {
                const int lm = i * 16 + lr;
                const int ln = wn * WN + j * 16 + lc;
                *(f4_t*)&Cs[lm * LDC4 + ln] = alpha * acc[i][j];
              }
          }
          __syncthreads();
          for (int c = tid; c < WM * CPR; c += NT) {
            const int row = c / CPR, col = (c % CPR) * EPC;
            const int64_t gm = m0 + pass * WM + row, gn = n0 + col;
            if (gm >= a.M) continue;
            if (a.cvec_ok && gn + EPC <= a.N) {
              *(uint4*)(dst + gm * ldd + gn) = *(const uint4*)(Cs + row * LDC4 + col);
            } else {
              for (int q = 0; q < EPC; ++q)
                if (gn + q < a.N) dst[gm * ldd + gn + q] = Cs[row * LDC4 + col + q];
            }
          }
          __syncthreads();
        }
      }
    } else {
  #pragma unroll
      for (int i = 0; i < TM; ++i)
  #pragma unroll
        for (int j = 0; j < TN; ++j)
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t gm = m0 + wm * WM + i * 16 + (lane & 15);
            const int64_t gn = n0 + wn * WN + j * 16 + 4 * (lane >> 4) + r;
            if (gm < a.M && gn < a.N) store_out<OutT>(a, tc, gm, gn, (double)acc[i][j][r]);
          }
    }
    if constexpr (!CHAIN) break;
    // the epilogue's LDS reads end before the next tile's first slice is stored
    if (more) __syncthreads();
    tc = tn;
  }
}

// ------------------------------------------------- short K, B in registers ----
// C = alpha A B^T for a k-contiguous BF16 A (M x K) and a BF16 B (N x K, k or n
// contiguous), with a short K (128, 256 or 384) and a BF16 result, batched,
// unsplit: the shape of Y = F^T B (one batch; K is a virtual dimension, N = X v
// runs to 10^5 and the M x N result is four times the size of B) and of
// Z = Y tau per r (R batches of X x v results from v x v operands).
//
// A work-group of eight waves owns 256 columns of one batch of C and a range of
// its rows (four waves and 128 columns at K = 384).
// Each wave loads the fragments of its 32 columns of B over the whole of K once
// (2 x K/32 fragments, 64 registers at K = 256; straight from memory when B is
// k-contiguous, else through LDS in 32-deep slabs with transposing reads) and
// keeps them for the work-group's life; blocks of 16 rows of A stream through
// LDS (two buffers, fed by a ring of register slots up to four blocks ahead
// while the matrix cores work on the current one), and each block's 16 x 256
// results are staged in LDS and written as whole 512-byte rows (stored straight
// from the accumulators, 32 bytes per row per instruction, they took twice as
// long as the products).
// B is thus read from HBM once, with no LDS traffic, and the pipeline runs over
// the rows instead of restarting every K = 256.
// (Blocks of 32 rows need more than the 128 registers of four waves per SIMD.)
// N must be a multiple of the work-group's columns and C 16-byte aligned with
// row and batch strides that are multiples of 8.
// Per fragment the arithmetic (one v_mfma_f32_16x16x32_bf16 per 32 k, in
// increasing k) is that of gemm_bf16_kernel, so both give the same bits.
// Offsets are 32-bit byte offsets from the operand bases (the launcher checks
// that they fit), which lets every load and store address a uniform base.
constexpr int RES_ROWS = 16;
// eight waves (256 columns, two work-groups per CU) for K = 128 and 256; four
// waves (128 columns, three per CU) for K = 384, whose 96 registers of B
// fragments leave room for three waves per SIMD only
constexpr int res_waves(int64_t K) { return K == 384 ? 4 : 8; }

struct ResArgs {
  const char* A;
  int64_t sam, sab;  // elements
  const char* B;
  int64_t sbn, sbk, sbb;  // one of sbn, sbk is 1
  const float* bscale;    // e4m3 B: per column (mode 1) or per k (mode 2)
  int bscale_mode;
  char* C;
  int64_t scm, scb;
  int64_t M, N;
  float alpha;
  int nblk;         // column blocks per batch
  int msplit;       // row ranges per column block
  int64_t mchunk;   // row blocks per row range
};

template <int KS, bool BKC, int WAVES, bool B8 = false>
__global__ __launch_bounds__(64 * WAVES, WAVES == 8 ? 4 : 3) void gemm_bf16_bres_kernel(const ResArgs r) {
  static_assert(!B8 || BKC, "an e4m3 B operand must be k-contiguous");
  constexpr int K = 32 * KS, CPR = K / 8, NT = 64 * WAVES;
  constexpr int RES_COLS = 32 * WAVES, CPRC = RES_COLS / 8;  // columns, 16-byte chunks per result row
  static_assert(RES_ROWS * CPRC == NT, "one result chunk per lane");
  constexpr int TC = RES_ROWS * CPR;          // 16-byte chunks of a row block
  constexpr int LPT = (TC + NT - 1) / NT;     // per lane (the last lanes idle if TC < NT)
  static_assert(TC % NT == 0 || TC < NT, "row block must divide over the lanes");
  constexpr int ABUF = RES_ROWS * K;        // bf16 per LDS buffer
  constexpr int CBUF = RES_ROWS * RES_COLS;  // bf16 per result staging buffer
  // a B stored with n contiguous is brought in 32-deep slabs through LDS
  using TB = BfTile<RES_COLS, false, 32, NT>;
  constexpr int SMEM_RUN = 2 * (2 * ABUF + 2 * CBUF), SMEM_B = BKC ? 0 : 2 * TB::SIZE;
  __shared__ __attribute__((aligned(16))) char smem[SMEM_RUN > SMEM_B ? SMEM_RUN : SMEM_B];
  bf16_t* const As = (bf16_t*)smem;
  bf16_t* const Cs = As + 2 * ABUF;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // each XCD takes a contiguous range of (batch, column block, row range)
  // triples, so the row ranges of one column block share its B in that XCD's L2
  const uint32_t G = gridDim.x;
  const uint32_t vid = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const uint32_t bn = vid / (uint32_t)r.msplit;
  const int64_t bt = bn / (uint32_t)r.nblk;
  const int64_t n0 = (int64_t)(bn % (uint32_t)r.nblk) * RES_COLS;
  const int64_t nrb = (r.M + RES_ROWS - 1) / RES_ROWS;
  const int64_t rb0 = (int64_t)(vid % (uint32_t)r.msplit) * r.mchunk;
  const int64_t rb1 = min(nrb, rb0 + r.mchunk);
  if (rb0 >= rb1) return;  // the whole work-group
  const char* const Ab = r.A + 2 * bt * r.sab;  // this batch's operands (uniform)
  const char* const Bb = r.B + 2 * bt * r.sbb;
  char* const Cb = r.C + 2 * bt * r.scb;

  // B fragments of this wave: lane l holds column n0 + 32 w + 16 ct + l % 16,
  // k = 32 ks + 8 (l / 16) .. + 7
  bf16x8_t bfr[2][KS];
  if constexpr (B8) {
    // e4m3 codes (one byte each, batch 0 only), decoded exactly and scaled
    // per column (mode 1) or per aligned group of 8 k (mode 2)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const uint32_t n = (uint32_t)(n0 + w * 32 + ct * 16 + (lane & 15));
      const uint32_t off = n * (uint32_t)r.sbn + 8u * (lane >> 4);
      const float sn = r.bscale_mode == 1 ? r.bscale[n] : 1.0f;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 q = *(const u32x2*)(r.B + (off + 32u * ks));
        const float sc = r.bscale_mode == 2 ? r.bscale[32 * ks + 8 * (lane >> 4)] : sn;
        bfr[ct][ks] = __builtin_bit_cast(bf16x8_t, e4m3x8_to_bf16(make_uint2(q[0], q[1]), sc));
      }
    }
  } else if constexpr (BKC) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const uint32_t n = (uint32_t)(n0 + w * 32 + ct * 16 + (lane & 15));
      const uint32_t off = 2u * (n * (uint32_t)r.sbn + 8u * (lane >> 4));
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) bfr[ct][ks] = *(const bf16x8_t*)(Bb + (off + 64u * ks));
    }
  } else {
    // slab ks: rows k = 32 ks .. + 31 of B (n contiguous, row stride sbk) as
    // [k][n] in LDS, then each wave's fragments by transposing reads
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      uint4 rb[TB::C];
      TB::template load<true>(rb, (const bf16_t*)Bb, 1, r.sbk, n0, n0 + RES_COLS, 32 * ks, K, true, tid);
      if (ks > 0) __syncthreads();  // the previous slab's fragment reads are done
      TB::store(rb, (bf16_t*)smem, tid);
      __syncthreads();
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) bfr[ct][ks] = TB::frag((const bf16_t*)smem, w * 32 + ct * 16, 0, lane);
    }
    __syncthreads();  // the slab region is reused by the row blocks
  }
  // Wait for them here: a first use inside the row loop would leave a wait for
  // every memory operation in flight (the next row block, the last block's
  // stores) in each trip.
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) asm volatile("" ::"v"(__builtin_bit_cast(u32x4, bfr[ct][ks])));

  // A row blocks: [16 rows][K] with the 16-byte chunk index XOR-ed with the
  // row, so that the 16 rows of a fragment read (one chunk each) and the 16
  // consecutive chunks of a row written by 16 lanes fall on distinct banks.
  // They come through a ring of P register slots, P blocks ahead of the one in
  // LDS.  Loads and stores retire in issue order, so waiting for a block's
  // load also waits for every store issued before it: with P slots, P - 1
  // trips' result stores stay in flight at that wait (one with two slots,
  // which held Y's stores to about 3 TB/s).  K = 384 keeps two slots: its
  // three loads per lane and slot would not fit in the registers left at
  // three waves per SIMD.
  constexpr int P = KS == 12 ? 2 : 4;
  uint4 ra[P][LPT];
  auto load_a = [&](uint4 (&slot)[LPT], int64_t rb) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < LPT; ++e) {
      const int c = tid + e * NT;
      if (TC < NT && c >= TC) break;
      const uint32_t g = (uint32_t)min(rb * RES_ROWS + c / CPR, r.M - 1);  // rows past M clamped
      slot[e] = load16((const bf16_t*)(Ab + 2u * (g * (uint32_t)r.sam + (uint32_t)(c % CPR) * 8u)));
    }
  };
  auto store_a = [&](const uint4 (&slot)[LPT], bf16_t* S) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < LPT; ++e) {
      const int c = tid + e * NT;
      if (TC < NT && c >= TC) break;
      const int row = c / CPR, ch = c % CPR;
      *(uint4*)&S[row * K + ((ch ^ row) << 3)] = slot[e];
    }
  };

  // Trip t computes row block min(rb0 + t, rb1 - 1): the trip count is padded
  // to a multiple of P and the padding trips recompute and store the last
  // block again (the same bits).  Every trip then runs the same memory
  // operations, and the compiler waits only for the block about to be written
  // to LDS.  Block t + 1 sits in slot (t + 1) % P and LDS buffer (t + 1) % 2.
  const int64_t last = rb1 - 1;
  load_a(ra[0], rb0);
  store_a(ra[0], As);
#pragma unroll
  for (int q = 1; q <= P; ++q) load_a(ra[q % P], min(rb0 + q, last));
  __syncthreads();
  const int lr = lane & 15;
  auto trip = [&](auto slot_c, int64_t t) __attribute__((always_inline)) {
    constexpr int S = decltype(slot_c)::value;  // t % P
    constexpr int cur = S & 1, nxt = (S + 1) % P;
    const int64_t rb = min(rb0 + t, last);
    const bf16_t* A_ = As + cur * ABUF;
    f4_t acc[2] = {f4_t{0.f, 0.f, 0.f, 0.f}, f4_t{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const bf16x8_t af = *(const bf16x8_t*)&A_[lr * K + (((ks * 4 + (lane >> 4)) ^ lr) << 3)];
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j][ks], af, acc[j], 0, 0, 0);
    }
    // Results to LDS (staging buffer cur, [16 rows][256 columns] with the
    // 16-byte chunk index XOR-ed with the row): lane l holds row l % 16,
    // columns 32 w + 16 j + 4 (l / 16) .. + 3.
    bf16_t* Cc = Cs + cur * CBUF;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = w * 32 + j * 16 + 4 * (lane >> 4);
      const uint32_t w0 = pack_bf16x2(r.alpha * acc[j][0], r.alpha * acc[j][1]);
      const uint32_t w1 = pack_bf16x2(r.alpha * acc[j][2], r.alpha * acc[j][3]);
      *(uint2*)&Cc[lr * RES_COLS + (((col >> 3) ^ lr) << 3) + (col & 7)] = make_uint2(w0, w1);
    }
    // LDS buffer cur ^ 1 was last read before the previous barrier
    store_a(ra[nxt], As + (cur ^ 1) * ABUF);
    load_a(ra[nxt], min(rb0 + t + 1 + P, last));
    __syncthreads();
    // Whole rows to memory: 16 bytes per lane, CPRC lanes per row.  (Staging
    // buffer cur is written again two trips on, after the next barrier.)  A row
    // past M was computed from the clamped last row of A, so it equals row
    // M - 1 and is stored there (the same bits twice).
    {
      const int row = tid / CPRC, ch = tid % CPRC;
      const uint32_t gm = (uint32_t)min(rb * RES_ROWS + row, r.M - 1);
      typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
      const u32x4 v = *(const u32x4*)&Cc[row * RES_COLS + ((ch ^ row) << 3)];
      __builtin_nontemporal_store(
          v, (u32x4*)(Cb + 2u * (gm * (uint32_t)r.scm + (uint32_t)n0 + 8u * ch)));
    }
  };
  auto group = [&](int64_t t0) __attribute__((always_inline)) {
    trip(std::integral_constant<int, 0>{}, t0);
    trip(std::integral_constant<int, 1>{}, t0 + 1);
    if constexpr (P == 4) {
      trip(std::integral_constant<int, 2>{}, t0 + 2);
      trip(std::integral_constant<int, 3>{}, t0 + 3);
    }
  };
  // The first group is peeled: in the loop the memory operations in flight at
  // the top are then always the next blocks' loads and the last trips' stores.
  const int64_t ntrip = (rb1 - rb0 + P - 1) / P * P;
  group(0);
  for (int64_t t0 = P; t0 < ntrip; t0 += P) group(t0);
}

// Sums the split-K partials in split order and applies alpha / beta.
template <typename PT, typename OutT>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const PT* __restrict__ part, int splits,
                                                            int64_t batch, int64_t M, int64_t N,
                                                            OutT* C, int64_t scm, int64_t scb,
                                                            double alpha, double beta) {
  const int64_t total = batch * M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    // loads in groups of eight so they are in flight together; the sum
    // still runs in split order
    double acc = 0.0;
    int s = 0;
    for (; s + 8 <= splits; s += 8) {
      PT v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = part[(s + q) * total + idx];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += (double)v[q];
    }
    for (; s < splits; ++s) acc += (double)part[s * total + idx];
    const int64_t b = idx / (M * N), rem = idx % (M * N);
    const int64_t m = rem / N, n = rem % N;
    OutT* c = C + b * scb + m * scm + n;
    double r = alpha * acc;
    if (beta != 0.0) r += beta * Conv<OutT>::to_f64(*c);
    *c = Conv<OutT>::from_f64(r);
  }
}

KArgs make_args(const Gemm& g, int BM, int BN, int BK) {
  KArgs a;
  a.M = g.M; a.N = g.N; a.K = g.K; a.batch = g.batch;
  a.A = g.A; a.sam = g.sam; a.sak = g.sak; a.sab = g.sab;
  a.B = g.B; a.sbk = g.sbk; a.sbn = g.sbn; a.sbb = g.sbb;
  a.C = g.C; a.scm = g.scm; a.scb = g.scb;
  a.alpha = g.alpha; a.beta = g.beta;
  int splits = std::max(1, g.splits);
  int64_t kchunk = (g.K + splits - 1) / splits;
  kchunk = std::max<int64_t>(BK, (kchunk + BK - 1) / BK * BK);
  splits = (int)std::max<int64_t>(1, (g.K + kchunk - 1) / kchunk);
  a.splits = splits;
  a.kchunk = g.K > 0 ? kchunk : 1;
  a.partial = g.partial;
  a.tiles_m = (g.M + BM - 1) / BM;
  a.tiles_n = (g.N + BN - 1) / BN;
  a.vec_ok = 0;
  a.cvec_ok = 0;
  a.bscale = g.bscale;
  a.bscale_mode = g.b_fp8 ? g.bscale_mode : 0;
  return a;
}

void check_operand_strides(const Gemm& g) {
  if (g.sak != 1 && g.sam != 1) throw std::invalid_argument("gemm: A has no unit stride");
  if (g.sbk != 1 && g.sbn != 1) throw std::invalid_argument("gemm: B has no unit stride");
  if (g.M < 0 || g.N < 0 || g.K < 0 || g.batch < 0) throw std::invalid_argument("gemm: negative size");
}

template <typename PT, typename OutT>
void launch_reduce(const KArgs& a, hipStream_t s) {
  const int64_t total = a.batch * a.M * a.N;
  int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL((splitk_reduce_kernel<PT, OutT>), dim3((unsigned)blocks), dim3(256), 0, s,
                     (const PT*)a.partial, a.splits, a.batch, a.M, a.N, (OutT*)a.C, a.scm, a.scb,
                     a.alpha, a.beta);
  CPPPL_LAUNCH_CHECK("splitk_reduce");
}

}  // namespace

int choose_splits(int64_t tiles, int64_t K, int64_t target_blocks, int64_t min_k, int max_splits) {
  if (tiles <= 0 || K <= 0) return 1;
  int64_t s = (target_blocks + tiles - 1) / tiles;
  s = std::min<int64_t>(s, std::max<int64_t>(1, K / std::max<int64_t>(1, min_k)));
  s = std::min<int64_t>(s, max_splits);
  return (int)std::max<int64_t>(1, s);
}

// Output tile rows of the FP64 kernel (64 columns): 128 when the problem is
// tall enough (each wave then owns 64 x 32 and issues twice the matrix-core
// work per staged slice), else 64.
static int f64_tile_m(int64_t M, int64_t N) { return (M >= 128 && N >= 64) ? 128 : 64; }
int64_t gemm_tiles_f64(int64_t M, int64_t N) {
  const int64_t t = f64_tile_m(M, N);
  return ((M + t - 1) / t) * ((N + 63) / 64);
}
// BF16 output tile rows: 256 (eight waves) for an unsplit product of two
// k-contiguous BF16 operands with K >= 1024, when M is a multiple of 256 of at
// least 512 or is at least 2048 (a ragged last tile row then wastes little);
// else 128.  Measured on MI355X, the 256-row tiles gain 2-11 % on such long-K
// products (the Khatri-Rao x t2 step) but lose 2-6 % on short K (v) and up to
// a third on split-K products, which keep 128 x 128 tiles with K slices of 64.
// (The transposing loads of row-contiguous operands would also need more
// registers than four waves per SIMD leave.)
static int bf16_tile_m(const Gemm& g) {
  const bool ok = g.sak == 1 && g.sbk == 1 && !g.b_fp8 && g.splits <= 1 && g.K >= 1024;
  return (ok && g.M >= 512 && (g.M % 256 == 0 || g.M >= 2048)) ? 256 : 128;
}
int64_t gemm_tiles_bf16(int64_t M, int64_t N) { return ((M + 127) / 128) * ((N + 127) / 128); }

template <int T>
static void launch_f64(const KArgs& a, bool ak, bool bk, dim3 grid, hipStream_t s) {
  dim3 block(256);
  if (ak && bk) hipLaunchKernelGGL((gemm_f64_kernel<T, 64, true, true>), grid, block, 0, s, a);
  else if (ak && !bk) hipLaunchKernelGGL((gemm_f64_kernel<T, 64, true, false>), grid, block, 0, s, a);
  else if (!ak && bk) hipLaunchKernelGGL((gemm_f64_kernel<T, 64, false, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gemm_f64_kernel<T, 64, false, false>), grid, block, 0, s, a);
}

int gemm_f64(const Gemm& g, hipStream_t s) {
  check_operand_strides(g);
  if (g.ctype != DType::F64) throw std::invalid_argument("gemm_f64: output must be FP64");
  int T = f64_tile_m(g.M, g.N);
  // a launch of fewer than 256 128-row work-groups leaves CUs idle: take
  // 64-row tiles instead (the R x R Gram products)
  if (T == 128) {
    const int64_t blocks128 = ((g.M + 127) / 128) * ((g.N + 63) / 64) * g.batch * std::max(1, g.splits);
    if (blocks128 < 256) T = 64;
  }
  KArgs a = make_args(g, T, 64, 16);
  if (a.splits > 1 && !a.partial) throw std::invalid_argument("gemm_f64: split-K needs a partial buffer");
  const int64_t blocks = a.tiles_m * a.tiles_n * a.batch * a.splits;
  if (blocks == 0) return a.splits;
  if (blocks > 0x7fffffffLL) throw std::invalid_argument("gemm_f64: grid too large");
  const bool ak = g.sak == 1, bk = g.sbk == 1;
  dim3 grid((unsigned)blocks);
  if (T == 128) launch_f64<128>(a, ak, bk, grid, s);
  else launch_f64<64>(a, ak, bk, grid, s);
  CPPPL_LAUNCH_CHECK("gemm_f64");
  if (a.splits > 1 && !g.keep_partials) launch_reduce<double, double>(a, s);
  return a.splits;
}

template <int BK, bool AK, bool BKC, bool B8 = false, int WGM = 2, bool FAST = false>
static void launch_bf16(const KArgs& a, DType ct, dim3 grid, hipStream_t s) {
  constexpr int BM = 64 * WGM, BN = 128;
  const dim3 block(128 * WGM);
  if (ct == DType::F32 || a.splits > 1)
    hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, BK, AK, BKC, float, B8, WGM, FAST>), grid, block, 0, s, a);
  else if (ct == DType::BF16)
    hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, BK, AK, BKC, bf16_t, B8, WGM, FAST>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, BK, AK, BKC, double, B8, WGM, FAST>), grid, block, 0, s, a);
}

template <int BK, bool FAST>
static void launch_bf16_layout(const KArgs& a, bool ak, bool bk, DType ct, dim3 grid,
                               hipStream_t s) {
  if (ak && bk) launch_bf16<BK, true, true, false, 2, FAST>(a, ct, grid, s);
  else if (ak && !bk) launch_bf16<BK, true, false, false, 2, FAST>(a, ct, grid, s);
  else if (!ak && bk) launch_bf16<BK, false, true, false, 2, FAST>(a, ct, grid, s);
  else launch_bf16<BK, false, false, false, 2, FAST>(a, ct, grid, s);
}

// About three rounds of work-groups at two per CU, each over at least eight
// row blocks.
static void launch_bres(const Gemm& g, hipStream_t s) {
  ResArgs r;
  r.A = (const char*)g.A; r.sam = g.sam; r.sab = g.sab;
  r.B = (const char*)g.B; r.sbn = g.sbn; r.sbk = g.sbk; r.sbb = g.sbb;
  r.bscale = g.bscale; r.bscale_mode = g.b_fp8 ? g.bscale_mode : 0;
  r.C = (char*)g.C; r.scm = g.scm; r.scb = g.scb;
  r.M = g.M; r.N = g.N;
  r.alpha = (float)g.alpha;
  const int waves = res_waves(g.K), res_cols = 32 * waves;
  const int64_t nblk = (g.N + res_cols - 1) / res_cols;
  const int64_t cols = nblk * g.batch;  // column blocks over all batches
  const int64_t nrb = (g.M + RES_ROWS - 1) / RES_ROWS;
  const int64_t target = 3 * 256 * (waves == 8 ? 2 : 3);  // three rounds of work-groups
  int64_t ms = std::max<int64_t>(1, std::min<int64_t>((target + cols - 1) / cols, nrb / 8));
  r.mchunk = (nrb + ms - 1) / ms;
  ms = (nrb + r.mchunk - 1) / r.mchunk;
  r.msplit = (int)ms;
  r.nblk = (int)nblk;
  const int64_t blocks = cols * ms;
  if (blocks > 0x7fffffffLL) throw std::invalid_argument("gemm_bf16: grid too large");
  const dim3 grid((unsigned)blocks), block(64 * waves);
  const bool bk = g.sbk == 1;
  if (g.b_fp8) {
    if (g.K == 384) hipLaunchKernelGGL((gemm_bf16_bres_kernel<12, true, 4, true>), grid, block, 0, s, r);
    else if (g.K == 256) hipLaunchKernelGGL((gemm_bf16_bres_kernel<8, true, 8, true>), grid, block, 0, s, r);
    else hipLaunchKernelGGL((gemm_bf16_bres_kernel<4, true, 8, true>), grid, block, 0, s, r);
  } else if (g.K == 384 && bk) hipLaunchKernelGGL((gemm_bf16_bres_kernel<12, true, 4>), grid, block, 0, s, r);
  else if (g.K == 384) hipLaunchKernelGGL((gemm_bf16_bres_kernel<12, false, 4>), grid, block, 0, s, r);
  else if (g.K == 256 && bk) hipLaunchKernelGGL((gemm_bf16_bres_kernel<8, true, 8>), grid, block, 0, s, r);
  else if (g.K == 256) hipLaunchKernelGGL((gemm_bf16_bres_kernel<8, false, 8>), grid, block, 0, s, r);
  else if (bk) hipLaunchKernelGGL((gemm_bf16_bres_kernel<4, true, 8>), grid, block, 0, s, r);
  else hipLaunchKernelGGL((gemm_bf16_bres_kernel<4, false, 8>), grid, block, 0, s, r);
  CPPPL_LAUNCH_CHECK("gemm_bf16 (B in registers)");
}

void gemm_bf16(const Gemm& g, hipStream_t s) {
  check_operand_strides(g);
  if (g.beta != 0.0 && g.splits <= 1) throw std::invalid_argument("gemm_bf16: beta must be 0");
  const bool ak = g.sak == 1, bk = g.sbk == 1;
  const int BM = bf16_tile_m(g), BN = 128;
  const int64_t kper = (g.K + std::max(1, g.splits) - 1) / std::max(1, g.splits);
  // 256-row tiles always walk K in short slices (their LDS stages are twice as large)
  const int bk_slice = (BM == 128 && kper >= BBK_LONG_MIN_K) ? BBK_LONG : BBK_SHORT;
  KArgs a = make_args(g, BM, BN, bk_slice);
  if (a.splits > 1 && !a.partial) throw std::invalid_argument("gemm_bf16: split-K needs a partial buffer");
  if (g.b_fp8) {
    if (!bk) throw std::invalid_argument("gemm_bf16: an e4m3 B must be k-contiguous");
    if (g.bscale_mode < 0 || g.bscale_mode > 2) throw std::invalid_argument("gemm_bf16: bad bscale_mode");
    if (g.bscale_mode != 0 && !g.bscale) throw std::invalid_argument("gemm_bf16: bscale is NULL");
  }
  // Vector loads need aligned rows along the contiguous index: 16 bytes for
  // 8 bfloat16, 8 bytes for 8 e4m3 codes.
  auto al = [](const void* p, uintptr_t b) { return ((uintptr_t)p & (b - 1)) == 0; };
  const int64_t sa_row = ak ? g.sam : g.sak, sb_row = bk ? g.sbn : g.sbk;
  a.vec_ok = (al(g.A, 16) && al(g.B, g.b_fp8 ? 8 : 16) && sa_row % 8 == 0 && sb_row % 8 == 0 &&
              g.sab % 8 == 0 && g.sbb % 8 == 0) ? 1 : 0;
  if (a.splits > 1) {
    a.cvec_ok = (al(g.partial, 16) && g.N % 4 == 0) ? 1 : 0;
  } else {
    const int64_t epc = g.ctype == DType::BF16 ? 8 : (g.ctype == DType::F32 ? 4 : 2);
    a.cvec_ok = (al(g.C, 16) && g.scm % epc == 0 && g.scb % epc == 0) ? 1 : 0;
  }
  const int64_t blocks = a.tiles_m * a.tiles_n * a.batch * a.splits;
  if (blocks == 0) return;
  if (blocks > 0x7fffffffLL) throw std::invalid_argument("gemm_bf16: grid too large");
  // unchecked loads when every slice is whole and every chunk aligned
  const bool fast = a.vec_ok && g.K > 0 && g.K % bk_slice == 0 && (ak || g.M % 8 == 0) &&
                    (bk || g.N % 8 == 0);
  // Short-K products of a few waves of work-groups, on 128 x 128 tiles at
  // four waves per SIMD, run two tiles per work-group, the second tile's
  // first slice loading before the first tile's results are stored.  Measured
  // on MI355X at o = 32, v = 256, X = 768, R = 1024 (Y and Z cut into launches
  // of 3072 tiles): the products alone ran as fast as with one tile per
  // work-group, but the ALS sweep ran 2-3 % faster, since side-stream inverse
  // steps are dispatched only once a launch's work-groups have all been
  // issued.  Other sizes measured worse: smaller grids leave CUs idle (3 %
  // slower at o = 16, v = 128), launches of 13824 tiles ran 1 % slower and
  // G's longer K (X = 1152) 10 % slower.  Without the early load the second
  // tile's loads queue behind the first tile's stores, and chained products
  // took twice as long.
  // Short-K products of a k-contiguous A over many columns with a BF16
  // result (Y = F^T B, Z = Y tau per r): B kept in registers, A streamed (see
  // gemm_bf16_bres_kernel).
  if ((!g.b_fp8 || (bk && g.batch == 1)) && ak && a.splits <= 1 && g.ctype == DType::BF16 &&
      (g.K == 128 || g.K == 256 || g.K == 384) && a.vec_ok && g.N % (32 * res_waves(g.K)) == 0 &&
      g.N * g.batch >= 16 * 32 * res_waves(g.K) && g.M >= 8 * RES_ROWS && ((uintptr_t)g.C & 15) == 0 &&
      g.scm % 8 == 0 && g.scb % 8 == 0 && g.sam >= g.K && g.N <= g.scm &&
      (bk ? g.sbn >= g.K : g.sbk >= g.N) && g.M * g.sam < (1LL << 31) &&
      (bk ? g.N * g.sbn : g.K * g.sbk) < (1LL << 31) && g.M * g.scm < (1LL << 31)) {
    launch_bres(g, s);
    return;
  }
  const bool four = (ak && bk) || (fast && !ak && !bk);
  const bool chain = fast && !g.b_fp8 && BM == 128 && bk_slice == BBK_SHORT && four &&
                     (g.ctype != DType::F64 || a.splits > 1) && blocks >= BF16_CHAIN_MIN_TILES &&
                     blocks <= BF16_CHAIN_MAX_TILES && a.kchunk <= BF16_CHAIN_MAX_K;
  dim3 grid((unsigned)(chain ? (blocks + 1) / 2 : blocks));
  if (g.b_fp8) {
    if (bk_slice == BBK_LONG) {
      if (ak && fast) launch_bf16<BBK_LONG, true, true, true, 2, true>(a, g.ctype, grid, s);
      else if (ak) launch_bf16<BBK_LONG, true, true, true>(a, g.ctype, grid, s);
      else if (fast) launch_bf16<BBK_LONG, false, true, true, 2, true>(a, g.ctype, grid, s);
      else launch_bf16<BBK_LONG, false, true, true>(a, g.ctype, grid, s);
    } else {
      if (ak && fast) launch_bf16<BBK_SHORT, true, true, true, 2, true>(a, g.ctype, grid, s);
      else if (ak) launch_bf16<BBK_SHORT, true, true, true>(a, g.ctype, grid, s);
      else if (fast) launch_bf16<BBK_SHORT, false, true, true, 2, true>(a, g.ctype, grid, s);
      else launch_bf16<BBK_SHORT, false, true, true>(a, g.ctype, grid, s);
    }
  } else {
    if (BM == 256) {
      if (fast) launch_bf16<BBK_SHORT, true, true, false, 4, true>(a, g.ctype, grid, s);
      else launch_bf16<BBK_SHORT, true, true, false, 4>(a, g.ctype, grid, s);
    } else if (bk_slice == BBK_LONG) {
      if (fast) launch_bf16_layout<BBK_LONG, true>(a, ak, bk, g.ctype, grid, s);
      else launch_bf16_layout<BBK_LONG, false>(a, ak, bk, g.ctype, grid, s);
    } else {
      if (fast) launch_bf16_layout<BBK_SHORT, true>(a, ak, bk, g.ctype, grid, s);
      else launch_bf16_layout<BBK_SHORT, false>(a, ak, bk, g.ctype, grid, s);
    }
  }
  CPPPL_LAUNCH_CHECK("gemm_bf16");
  if (a.splits > 1) {
    if (g.ctype == DType::F32) launch_reduce<float, float>(a, s);
    else if (g.ctype == DType::BF16) launch_reduce<float, bf16_t>(a, s);
    else launch_reduce<float, double>(a, s);
  }
}

}  // namespace cpppl
