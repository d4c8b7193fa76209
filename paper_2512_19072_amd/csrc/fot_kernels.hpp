// Device code of the FOT library for gfx950 (CDNA4), apart from the fused iteration kernels.
//
// The iteration loop of Algorithm 1 (arXiv 2512.19072, Sec. 3) runs in fot_fused.hpp.  This file
// holds what the solve needs around it:
//   * element conversions to the operand types and the MFMA traits (16 x 16 tiles; fragment
//     layouts and accumulator row maps) shared with the fused kernels;
//   * a general MFMA GEMM C = A . B^T (both operands K-contiguous, 64 x 64 output tiles) for the
//     once-per-solve FP64 products: the read-out of the final potentials (ln S, the phase moments
//     of Eq. 9-10, the transport cost) and the DFT of the output beam.  Its operands are shifted
//     per row (k_rowexp) before the first product and per column (k_colexpT) before the second
//     (the reverse sweep's signed contractions run on the fused kernels); the column maxima are gathered
//     across workgroups with atomicMax on order-preserving integer keys of their FP32 roundings
//     (a shift only has to keep the sums in range, so its rounding does not matter).  Lambda and
//     Lambda o H, functions of the pixel distance alone, enter it as Toeplitz chunk tables (a few
//     KB, read through the caches) instead of n_p x n_p planes;
//   * set-up kernels (row sums of the squared amplitudes, ln a and ln b, Lambda, initial
//     potentials), the read-out's reductions (k_readout, one launch per pass-2 moment, k_colerr,
//     and k_sum_parts: fixed-order partial sums),
//     the trapezoid integration of the phase, and the reverse sweep's elementwise kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

namespace fot {

constexpr int TILE = 64;          // output tile edge of one workgroup
constexpr int NTHREADS = 256;     // 4 wave64s, each owning a 32 x 32 quarter of the tile
constexpr int ROWB = 256;         // bytes of one operand row per K stage
constexpr int LDS_RS = ROWB + 16; // LDS row stride in bytes (16 B of padding: conflict-free b128 reads)
constexpr int CHUNKS = ROWB / 16; // 16-byte chunks per operand row per stage

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // one 16-byte fragment

// ------------------------------------------------------------------ element conversions
template <typename T> __device__ __forceinline__ T from_float(float x);
template <> __device__ __forceinline__ float from_float<float>(float x) { return x; }
template <> __device__ __forceinline__ __bf16 from_float<__bf16>(float x) { return (__bf16)x; }
template <> __device__ __forceinline__ _Float16 from_float<_Float16>(float x) { return (_Float16)x; }

// BF16x3 operands: a value v is held as hi = bf16(v) and lo = bf16(v - hi), both rounded to
// nearest even, so hi + lo carries about 16 significant bits with BF16's (= FP32's) exponent
// range.  A product of two such operands is formed as hi.hi + hi.lo + lo.hi by three BF16
// MFMAs into one FP32 accumulator; the dropped lo.lo term is below 2^-16 of the product.
// In memory an operand row of np values takes 2 np BF16 (4 bytes per value, like FP32):
// each group of 32 consecutive values is stored as its 32 hi halves, then its 32 lo halves,
// so one 64-byte fragment step of the GEMM reads either the hi or the lo halves of 32 values
// and the MFMA loop needs no repacking.  The struct is the element type of the API (its size
// sets the row pitch); it is not the memory layout.
struct bf16x3 {
  __bf16 hi, lo;
};
template <> __device__ __forceinline__ bf16x3 from_float<bf16x3>(float x) {
  const __bf16 h = (__bf16)x;
  return bf16x3{h, (__bf16)(x - (float)h)};   // x - hi is exact in FP32
}

// a double rounded to the operand type (BF16x3: split from the double itself)
template <typename T> __device__ __forceinline__ T cvt_op(double v) { return (T)v; }
template <> __device__ __forceinline__ bf16x3 cvt_op<bf16x3>(double v) {
  const __bf16 h = (__bf16)v;
  return bf16x3{h, (__bf16)(v - (double)h)};
}

// element k of an operand row that starts at `row` (np elements of T)
template <typename T> __device__ __forceinline__ void store_op(T* row, int k, T v) { row[k] = v; }
template <> __device__ __forceinline__ void store_op<bf16x3>(bf16x3* row, int k, bf16x3 v) {
  __bf16* r = (__bf16*)row + 2 * (k & ~31) + (k & 31);
  r[0] = v.hi;
  r[32] = v.lo;
}

// exp of a non-positive log-weight, rounded to the operand type.  FP64 operands use the
// FP64 exponential; the others evaluate expf on the FP32-rounded argument (the argument is
// <= 0 and near 0 for the entries that matter, so its rounding is harmless).
template <typename T> __device__ __forceinline__ T exp_op(double x) {
  return from_float<T>(expf((float)x));
}
template <> __device__ __forceinline__ double exp_op<double>(double x) { return exp(x); }

// w * exp(x), rounded once to the operand type.
template <typename T> __device__ __forceinline__ T scaled_exp_op(double x, double w) {
  return from_float<T>(expf((float)x) * (float)w);
}
template <> __device__ __forceinline__ double scaled_exp_op<double>(double x, double w) { return exp(x) * w; }

template <typename T> __device__ __forceinline__ T signed_exp_op(double mag_log, bool neg) {
  T v = exp_op<T>(mag_log);
  return neg ? (T)(-v) : v;
}

// ------------------------------------------------------------------ ordered float keys
// Column maxima across workgroups use atomicMax on an order-preserving encoding of float.
// Key 0 means "no finite value seen" (it decodes to no shift).
__device__ __forceinline__ unsigned float_key(float f) {
  unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ double key_to_shift(unsigned key) {
  if (key == 0u) return 0.0;
  unsigned u = (key & 0x80000000u) ? (key & 0x7fffffffu) : ~key;
  float f = __uint_as_float(u);
  return (f > -INFINITY && f < INFINITY) ? (double)f : 0.0;
}

// ------------------------------------------------------------------ MFMA traits
// One 16-byte LDS fragment per lane holds 16/sizeof(T) consecutive K elements.  A and B
// fragments use the same K mapping, so the products pair up correctly whatever order the
// instruction assigns to K inside the fragment.
template <typename T> struct Mma;

// Output layout of the 16 x 16 accumulator: lane l holds column l % 16; register e holds
// row row(l / 16, e).  FP32/BF16/FP16 blocks are 4 consecutive rows per lane group, FP64
// rows are interleaved with stride 4 (checked by the GEMM parity tests).
template <> struct Mma<float> {
  typedef f32x4 acc_t;
  typedef float out_t;
  static __device__ __forceinline__ int row(int g, int e) { return 4 * g + e; }
  static __device__ __forceinline__ void run(const u32x4& a, const u32x4& b, acc_t& c) {
    const f32x4 av = __builtin_bit_cast(f32x4, a);
    const f32x4 bv = __builtin_bit_cast(f32x4, b);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0], bv[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1], bv[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2], bv[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[3], bv[3], c, 0, 0, 0);
  }
  // the q-th of run's NSUB products (callers interleave accumulators between them)
  static constexpr int NSUB = 4;
  static constexpr bool PAIRED = false;
  static __device__ __forceinline__ void sub(const u32x4& a, const u32x4& b, acc_t& c, int q) {
    const f32x4 av = __builtin_bit_cast(f32x4, a);
    const f32x4 bv = __builtin_bit_cast(f32x4, b);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv[q], c, 0, 0, 0);
  }
};

template <> struct Mma<double> {
  typedef f64x4 acc_t;
  typedef double out_t;
  static __device__ __forceinline__ int row(int g, int e) { return g + 4 * e; }
  static __device__ __forceinline__ void run(const u32x4& a, const u32x4& b, acc_t& c) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 av = __builtin_bit_cast(d2, a);
    const d2 bv = __builtin_bit_cast(d2, b);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], bv[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], bv[1], c, 0, 0, 0);
  }
  static constexpr int NSUB = 2;
  static constexpr bool PAIRED = false;
  static __device__ __forceinline__ void sub(const u32x4& a, const u32x4& b, acc_t& c, int q) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(__builtin_bit_cast(d2, a)[q], __builtin_bit_cast(d2, b)[q], c, 0, 0, 0);
  }
};

template <> struct Mma<__bf16> {
  typedef f32x4 acc_t;
  typedef float out_t;
  static __device__ __forceinline__ int row(int g, int e) { return 4 * g + e; }
  static __device__ __forceinline__ void run(const u32x4& a, const u32x4& b, acc_t& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
  static constexpr int NSUB = 1;
  static constexpr bool PAIRED = false;
  static __device__ __forceinline__ void sub(const u32x4& a, const u32x4& b, acc_t& c, int) { run(a, b, c); }
};

// BF16x3: fragment steps come in pairs, the hi halves of 32 K values and then their lo halves
// (the fused GEMM issues hi.hi on the first step of a pair and hi.lo, lo.hi on the second)
template <> struct Mma<bf16x3> : Mma<__bf16> {
  static constexpr bool PAIRED = true;
};

template <> struct Mma<_Float16> {
  typedef f32x4 acc_t;
  typedef float out_t;
  static __device__ __forceinline__ int row(int g, int e) { return 4 * g + e; }
  static __device__ __forceinline__ void run(const u32x4& a, const u32x4& b, acc_t& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                               __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  }
  static constexpr int NSUB = 1;
  static constexpr bool PAIRED = false;
  static __device__ __forceinline__ void sub(const u32x4& a, const u32x4& b, acc_t& c, int) { run(a, b, c); }
};

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block-wide sum of one double per thread in a fixed order (deterministic).
__device__ __forceinline__ double block_sum(double v, double* scratch /* >= 4 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) s += scratch[w];
  return s;
}
__device__ __forceinline__ double block_max(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double s = -INFINITY;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) s = fmax(s, scratch[w]);
  return s;
}

// ------------------------------------------------------------------ GEMM (C = A . B^T)
enum Epilogue { EPI_LOGROW = 0, EPI_RAW = 2 };

struct GemmArgs {
  const void* A;            // [batch][np][np] (row i, K contiguous); sA = 0 shares it
  const void* B;            // [batch][np][np] (row j, K contiguous)
  long long sA, sB;         // batch strides in elements
  int n, np, nk;            // valid size, padded size, number of K stages
  int xcd_swizzle;          // remap workgroups so each XCD works on a compact block of tiles
  int kp;                   // row pitch of A and B in elements (0: np); the K extent is nk stages
  int ldo;                  // EPI_RAW: row pitch of the output in elements (0: np)
  // or nullptr: the operand is Lambda-like (its entry (r, k) a function of |r - k| alone) and is read
  // from that function's Toeplitz chunks instead of A / B: chunk c holds the 16 / sizeof(T) values
  // at distances c - (np - 1), c - (np - 1) + 1, ... (2 np chunks, see k_lam_table64); row pitch np
  const void* tzA;
  const void* tzB;
  // EPI_LOGROW / EPI_RAW output (Z type, [batch][np][ldo])
  void* out;
  long long sOut;
  const double* mrow;       // [batch][np] row shifts of the pass-1 operand
  unsigned* colkey;         // [batch][np] column-max keys (pass 1 writes, pass 2 reads)
};

// Map the linear workgroup id to a tile so that the workgroups that land on one XCD
// (hardware round-robin: id % 8) share operand panels in that XCD's L2.  swz = XCD_BLOCKS: a
// compact block of tiles that shares A rows and B columns; XCD_ROWS / XCD_COLS: whole bands of
// tile rows / tile columns, for products whose B / A operand (Lambda's Toeplitz table) is not a
// panel, so that each panel of the other operand is fetched by one XCD.
enum { XCD_NONE = 0, XCD_BLOCKS = 1, XCD_ROWS = 2, XCD_COLS = 3 };
__device__ __forceinline__ void tile_of(int tiles_x, int tiles_y, int swz, int* tr, int* tc) {
  const int total = tiles_x * tiles_y;
  int w = blockIdx.x + tiles_x * blockIdx.y;
  if (swz && (total % 8) == 0) {
    const int per = total / 8;
    w = (w % 8) * per + (w / 8);
  }
  if (swz == XCD_ROWS) {
    *tr = w / tiles_x;
    *tc = w % tiles_x;
    return;
  }
  if (swz == XCD_COLS) {
    *tc = w / tiles_y;
    *tr = w % tiles_y;
    return;
  }
  const int GROUP = 4;
  const int per_group = GROUP * tiles_x;
  const int grp = w / per_group;
  const int first = grp * GROUP;
  const int gsz = min(tiles_y - first, GROUP);
  const int in = w % per_group;
  *tr = first + in % gsz;
  *tc = in / gsz;
}

// Tile configuration: a BM x BN output tile per workgroup of NW wave64s; every wave owns an
// (RB*16) x (CB*16) block of 16 x 16 MFMA tiles.  The fused kernels normalise their operands in
// exponent blocks of BN / XS (pass-1 operand) and BM / XS (pass-2 operand) K values.
template <int BM_, int BN_, int NW_, int RB_, int CB_, int XS_ = 1>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, NW = NW_, RB = RB_, CB = CB_, XS = XS_;
  static constexpr int WTM = 16 * RB, WTN = 16 * CB;          // wave tile
  static constexpr int WGN = BN / WTN, WGM = BM / WTM;         // waves along N and M
  static constexpr int THREADS = 64 * NW;
  static_assert(WGN * WGM == NW, "waves must tile the workgroup tile");
  static_assert((BM * CHUNKS) % THREADS == 0 && (BN * CHUNKS) % THREADS == 0, "loads must divide");
};
typedef Cfg<64, 64, 4, 2, 2> Cfg64x64w4;
typedef Cfg<64, 64, 8, 2, 1> Cfg64x64w8;
typedef Cfg<64, 32, 4, 2, 1> Cfg64x32w4;

template <typename T, int EPI, typename C>
__global__ __launch_bounds__(C::THREADS) void k_gemm(const GemmArgs p) {
  typedef typename Mma<T>::acc_t acc_t;
  typedef typename Mma<T>::out_t zt;           // float, or double for FP64
  constexpr int BM = C::BM, BN = C::BN, RB = C::RB, CB = C::CB;
  __shared__ __attribute__((aligned(16))) unsigned char ldsA[2][BM * LDS_RS];
  __shared__ __attribute__((aligned(16))) unsigned char ldsB[2][BN * LDS_RS];
  __shared__ float cmax[C::WGM][BN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / C::WGN, wn = wave % C::WGN;
  const int r16 = lane & 15, g = lane >> 4;
  const int bz = blockIdx.z;
  int tr, tc;
  tile_of(gridDim.x, gridDim.y, p.xcd_swizzle, &tr, &tc);
  const int row0 = tr * BM, col0 = tc * BN;
  const size_t pitch = (size_t)(p.kp ? p.kp : p.np) * sizeof(T);
  const unsigned char* Ab = (const unsigned char*)p.A + ((size_t)bz * p.sA) * sizeof(T) + (size_t)row0 * pitch;
  const unsigned char* Bb = (const unsigned char*)p.B + ((size_t)bz * p.sB) * sizeof(T) + (size_t)col0 * pitch;

  // each thread moves LA (LB) 16-byte chunks of A (B) per K stage, kept in registers while
  // the previous stage is consumed
  constexpr int LA = BM * CHUNKS / C::THREADS, LB = BN * CHUNKS / C::THREADS;
  constexpr int RSTEP = C::THREADS / CHUNKS;      // rows covered by one pass of the block
  const int rl = tid / CHUNKS, ql = tid % CHUNKS;
  const unsigned char* Ag = Ab + (size_t)rl * pitch + (size_t)ql * 16;
  const unsigned char* Bg = Bb + (size_t)rl * pitch + (size_t)ql * 16;
  const int sofs = rl * LDS_RS + ql * 16;
  u32x4 ga[LA], gb[LB];
  // chunk u of stage kt: row rl + u RSTEP of the tile, K values from kt KPS + ql EPC; a Toeplitz
  // operand's row r holds at K the value at distance K - r, i.e. chunk K - r + np - 1 of its table
  constexpr int KPS = ROWB / (int)sizeof(T), EPC = 16 / (int)sizeof(T);
  const int tz0 = ql * EPC - rl + p.np - 1;
  auto load_a = [&](int u, int kt) -> u32x4 {
    if (p.tzA) return ((const u32x4*)p.tzA)[tz0 + kt * KPS - row0 - u * RSTEP];
    return *(const u32x4*)(Ag + (size_t)u * RSTEP * pitch + (size_t)kt * ROWB);
  };
  auto load_b = [&](int u, int kt) -> u32x4 {
    if (p.tzB) return ((const u32x4*)p.tzB)[tz0 + kt * KPS - col0 - u * RSTEP];
    return *(const u32x4*)(Bg + (size_t)u * RSTEP * pitch + (size_t)kt * ROWB);
  };

  acc_t acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = acc_t{};
  // FP32 accumulators are flushed into FP64 running sums after every K stage, so rounding
  // grows with the 64-128 products of one stage rather than with the whole K extent.
  constexpr bool FLUSH = sizeof(typename Mma<T>::out_t) == 4;
  f64x4 accd[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) accd[i][j] = f64x4{};

#pragma unroll
  for (int u = 0; u < LA; ++u) ga[u] = load_a(u, 0);
#pragma unroll
  for (int u = 0; u < LB; ++u) gb[u] = load_b(u, 0);
#pragma unroll
  for (int u = 0; u < LA; ++u) *(u32x4*)(&ldsA[0][sofs + u * RSTEP * LDS_RS]) = ga[u];
#pragma unroll
  for (int u = 0; u < LB; ++u) *(u32x4*)(&ldsB[0][sofs + u * RSTEP * LDS_RS]) = gb[u];
  __syncthreads();
  for (int kt = 0; kt < p.nk; ++kt) {
    const int s = kt & 1;
    const bool more = kt + 1 < p.nk;
    if (more) {
#pragma unroll
      for (int u = 0; u < LA; ++u) ga[u] = load_a(u, kt + 1);
#pragma unroll
      for (int u = 0; u < LB; ++u) gb[u] = load_b(u, kt + 1);
    }
#pragma unroll
    for (int h = 0; h < CHUNKS / 4; ++h) {
      u32x4 af[RB], bf[CB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
        af[rb] = *(const u32x4*)(&ldsA[s][(wm * C::WTM + rb * 16 + r16) * LDS_RS + (h * 4 + g) * 16]);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
        bf[cb] = *(const u32x4*)(&ldsB[s][(wn * C::WTN + cb * 16 + r16) * LDS_RS + (h * 4 + g) * 16]);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) Mma<T>::run(af[rb], bf[cb], acc[rb][cb]);
    }
    if constexpr (FLUSH) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
          for (int e = 0; e < 4; ++e) accd[rb][cb][e] += (double)acc[rb][cb][e];
          acc[rb][cb] = acc_t{};
        }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < LA; ++u) *(u32x4*)(&ldsA[s ^ 1][sofs + u * RSTEP * LDS_RS]) = ga[u];
#pragma unroll
      for (int u = 0; u < LB; ++u) *(u32x4*)(&ldsB[s ^ 1][sofs + u * RSTEP * LDS_RS]) = gb[u];
    }
    __syncthreads();
  }

  // ---------------------------------------------------------------- epilogues
  // result(rb, cb, e) is C[row0 + wm*WTM + rb*16 + Mma<T>::row(g, e)][col0 + wn*WTN + cb*16 + r16]
  auto result = [&](int rb, int cb, int e) -> double {
    if constexpr (FLUSH)
      return accd[rb][cb][e];
    else
      return (double)acc[rb][cb][e];
  };
  // ln of a result (the FP32 output of FP32/16-bit operands is stored rounded anyway)
  auto log_result = [&](int rb, int cb, int e) -> double {
    if constexpr (FLUSH)
      return (double)logf((float)accd[rb][cb][e]);
    else
      return log((double)acc[rb][cb][e]);
  };
  const int n = p.n, np = p.np;
  if constexpr (EPI == EPI_RAW) {
    zt* out = (zt*)p.out + (size_t)bz * p.sOut;
    const size_t ldo = p.ldo ? (size_t)p.ldo : (size_t)np;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = row0 + wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const int j = col0 + wn * C::WTN + cb * 16 + r16;
          if (i < n && j < n) out[(size_t)i * ldo + j] = (zt)result(rb, cb, e);
        }
  } else if constexpr (EPI == EPI_LOGROW) {
    zt* out = (zt*)p.out + (size_t)bz * p.sOut;
    const double* mrow = p.mrow + (size_t)bz * np;
    double cm[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) cm[cb] = -INFINITY;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = row0 + wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const int j = col0 + wn * C::WTN + cb * 16 + r16;
          if (i < n && j < n) {
            const zt z = (zt)log_result(rb, cb, e);
            out[(size_t)i * np + j] = z;
            cm[cb] = fmax(cm[cb], mrow[i] + (double)z);
          }
        }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      cm[cb] = fmax(cm[cb], __shfl_xor(cm[cb], 16, 64));
      cm[cb] = fmax(cm[cb], __shfl_xor(cm[cb], 32, 64));
      if (g == 0) cmax[wm][wn * C::WTN + cb * 16 + r16] = (float)cm[cb];
    }
    __syncthreads();
    if (tid < BN) {
      float m = cmax[0][tid];
#pragma unroll
      for (int w = 1; w < C::WGM; ++w) m = fmaxf(m, cmax[w][tid]);
      const int j = col0 + tid;
      if (j < n && m > -INFINITY) atomicMax(p.colkey + (size_t)bz * np + j, float_key(m));
    }
  }
}

// ------------------------------------------------------------------ operand preparation
// Row shift and shifted exponentials of a potential (pass-1 operand):
//   m_i = max_k P_ik / eps (0 if the row has no finite entry), out_ik = exp(P_ik/eps - m_i).
// Optionally out2_ik = out_ik * Y_k with Y_k = (k - floor(n/2)) / sqrt(n) (Eq. 10 moment).
// Also clears the column-max keys that the following pass 1 fills (unless colkey is null: then out is
// rewritten with the same values and the keys stay).  With out = nullptr only out2 is written (the
// same values), and the row shifts and column keys are left as they are.
//
// Block 0 of each batch entry also finishes the marginal-error reduction of the preceding
// potential update: red_out[bz] = sum of red_parts[bz][0..red_tiles) in index order.
struct PendingSum {
  const double* parts;   // nullptr: nothing pending
  int tiles;
  double* out;           // [batch]
};

__device__ __forceinline__ void finish_pending(const PendingSum& ps, int bz, double* red) {
  double v = 0.0;
  for (int t = threadIdx.x; t < ps.tiles; t += blockDim.x) v += ps.parts[(size_t)bz * ps.tiles + t];
  v = block_sum(v, red);
  if (threadIdx.x == 0) ps.out[bz] = v;
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_rowexp(const double* P, int n, int np, double inv_eps,
                                                     double* mrow, T* out, T* out2, unsigned* colkey,
                                                     const PendingSum pend) {
  constexpr int MAXV = 32;  // n <= 8192 = 32 * NTHREADS
  __shared__ double red[4];
  const int i = blockIdx.x, bz = blockIdx.y;
  if (i == 0 && pend.parts) finish_pending(pend, bz, red);
  const size_t plane = (size_t)np * np;
  T* o = out ? out + bz * plane + (size_t)i * np : nullptr;
  T* o2 = out2 ? out2 + bz * plane + (size_t)i * np : nullptr;
  if (o && colkey && threadIdx.x == 0) colkey[(size_t)bz * np + i] = 0u;
  if (i >= n) {
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
      if (o) o[k] = (T)0;
      if (o2) o2[k] = (T)0;
    }
    if (o && threadIdx.x == 0) mrow[(size_t)bz * np + i] = 0.0;
    return;
  }
  const double* row = P + bz * plane + (size_t)i * np;
  const int cnt = (n + NTHREADS - 1) / NTHREADS;   // np <= cnt * NTHREADS as well
  double v[MAXV];
  double m = -INFINITY;
#pragma unroll
  for (int c = 0; c < MAXV; ++c) {
    if (c < cnt) {
      const int k = threadIdx.x + c * NTHREADS;
      v[c] = (k < n) ? row[k] * inv_eps : -INFINITY;
      m = fmax(m, v[c]);
    }
  }
  m = block_max(m, red);
  if (!(m > -INFINITY && m < INFINITY)) m = 0.0;
  if (o && threadIdx.x == 0) mrow[(size_t)bz * np + i] = m;
  const double ysc = 1.0 / sqrt((double)n);
#pragma unroll
  for (int c = 0; c < MAXV; ++c) {
    if (c < cnt) {
      const int k = threadIdx.x + c * NTHREADS;
      if (k < np) {
        const bool ok = k < n;
        if (o) o[k] = ok ? exp_op<T>(v[c] - m) : (T)0;
        if (o2) o2[k] = ok ? scaled_exp_op<T>(v[c] - m, (double)(k - n / 2) * ysc) : (T)0;
      }
    }
  }
}

// Pass-2 operand, transposed: outT[k][L] = weight * exp(m_L - m'_k) * W[L][k] where
//   MODE 0: Z = ln W (from EPI_LOGROW), weight 1
//   MODE 1: Z = ln W, weight X_L = (L - floor(n/2)) / sqrt(n)   (Eq. 9 moment)
//   MODE 2: Z = W itself (signed, from EPI_RAW), weight 1
template <typename T, typename ZT, int MODE>
__global__ __launch_bounds__(NTHREADS) void k_colexpT(const ZT* Z, const double* mrow, const unsigned* colkey,
                                                      int n, int np, T* outT) {
  // each thread transposes a 4 x 4 block: rows L0..L0+3 of Z, columns k0..k0+3
  typedef ZT zv4 __attribute__((ext_vector_type(4)));
  typedef T tv4 __attribute__((ext_vector_type(4)));
  const int bz = blockIdx.z;
  const int L0 = blockIdx.y * TILE + 4 * (threadIdx.x >> 4);
  const int k0 = blockIdx.x * TILE + 4 * (threadIdx.x & 15);
  const size_t plane = (size_t)np * np;
  const double xsc = 1.0 / sqrt((double)n);
  double mk[4], ml[4];
  zv4 z[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    mk[i] = (k0 + i < n) ? key_to_shift(colkey[(size_t)bz * np + k0 + i]) : 0.0;
    ml[i] = (L0 + i < n) ? mrow[(size_t)bz * np + L0 + i] : 0.0;
    z[i] = *(const zv4*)(Z + bz * plane + (size_t)(L0 + i) * np + k0);
  }
  tv4 out[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      T v = (T)0;
      if (L0 + i < n && k0 + j < n) {
        const double zz = (double)z[i][j];
        if (MODE == 2) {
          v = (zz == 0.0) ? (T)0 : signed_exp_op<T>(log(fabs(zz)) + (ml[i] - mk[j]), zz < 0.0);
        } else if (MODE == 1) {
          v = scaled_exp_op<T>((ml[i] - mk[j]) + zz, (double)(L0 + i - n / 2) * xsc);
        } else {
          v = exp_op<T>((ml[i] - mk[j]) + zz);
        }
      }
      out[j][i] = v;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) *(tv4*)(outT + bz * plane + (size_t)(k0 + j) * np + L0) = out[j];
}

// Gibbs factor Lambda[i][k] = exp(-(i-k)^2 / (2 n^2 eps)) (Sec. 3, after Eq. 6), optionally
// times the axis cost H = (i-k)^2 / (2 n^2) for the transport-cost moments.  Padded rows and
// columns are filled by the same formula; they only ever meet zero operands.
template <typename T>
__global__ void k_fill_lambda(T* lam, T* lamH, int n, int np, double inv_eps) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int i = (int)(idx / np), k = (int)(idx % np);
  const double d = (double)(i - k);
  const double h = d * d / (2.0 * (double)n * (double)n);
  const double v = exp(-h * inv_eps);
  store_op<T>(lam + (size_t)i * np, k, cvt_op<T>(v));
  if (lamH) store_op<T>(lamH + (size_t)i * np, k, cvt_op<T>(v * h));
}

// The same two functions of the distance d = i - k in FP64 as Toeplitz chunks (the form k_gemm
// reads through GemmArgs::tzA / tzB): chunk c holds the values at d = c - (np - 1) and d + 1, zero
// where |d| >= np; element for element equal to the planes k_fill_lambda writes.  One thread per
// chunk; either table may be null.
__global__ void k_lam_table64(double* tz, double* tzH, int n, int np, double inv_eps) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 2 * np) return;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int di = c - (np - 1) + e;
    const double d = (double)di;
    const double h = d * d / (2.0 * (double)n * (double)n);
    const double v = exp(-h * inv_eps);
    const bool in = di < np && di > -np;
    if (tz) tz[2 * c + e] = in ? v : 0.0;
    if (tzH) tzH[2 * c + e] = in ? v * h : 0.0;
  }
}

// ------------------------------------------------------------------ marginals (Eq. 2)
// Row sums of squared amplitudes (one block per row), with input validation.
__global__ void k_rowsumsq(const double* x, int n, double* rowsum, int* flag) {
  __shared__ double red[4];
  const int i = blockIdx.x, bz = blockIdx.y;
  const double* row = x + ((size_t)bz * n + i) * n;
  double s = 0.0;
  int bad = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double v = row[k];
    bad |= !(v >= 0.0 && v < INFINITY);
    s += v * v;
  }
  if (bad) atomicOr(flag, 2);
  s = block_sum(s, red);
  if (threadIdx.x == 0) rowsum[(size_t)bz * n + i] = s;
}

// ln of the normalised intensity x^2 / sum x^2 into the padded layout (-inf at zeros and
// in the padding).  Every block re-sums the row sums in the same order.
__global__ void k_logmarg(const double* x, const double* rowsum, int n, int np, double* lnm, int* flag) {
  __shared__ double red[4];
  const int i = blockIdx.x, bz = blockIdx.y;
  double t = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x) t += rowsum[(size_t)bz * n + r];
  t = block_sum(t, red);
  if (!(t > 0.0 && t < INFINITY)) {
    if (threadIdx.x == 0) atomicOr(flag, 4);
    t = 1.0;
  }
  const double lt = log(t);
  double* o = lnm + ((size_t)bz * np + i) * np;
  for (int k = threadIdx.x; k < np; k += blockDim.x) {
    double v = -INFINITY;
    if (i < n && k < n) {
      const double a = x[((size_t)bz * n + i) * n + k];
      if (a > 0.0) v = 2.0 * log(a) - lt;
    }
    o[k] = v;
  }
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_fill_pot(double* pot, int n, int np, int batch, double value) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t plane = (size_t)np * np;
  if (idx >= plane * batch) return;
  const size_t r = idx % plane;
  const int i = (int)(r / np), k = (int)(r % np);
  pot[idx] = (i < n && k < n) ? value : -INFINITY;
}

// ln S from a raw pass-2 output: ln S = m'_k + ln S~ (-inf where S~ = 0), valid pixels only.
// ------------------------------------------------------------------ read-out (Eq. 9-10)
// The read-out's pass-2 outputs M are formed one at a time and each is consumed by one launch of
// k_readout<ROLE>.  M is the output for V_T divided by exp(m'_k); u/a = 1/S_prev with
// ln S_prev = ln(Lambda V_{T-1} Lambda) from the final u-update, so that a pixel's factor is
// scale = exp(m'_k - ln S_prev).  Roles:
//   RO_S:   M = S.  Per-block partial sums of |row mass - a| (slot 0), the row mass (1),
//           <f,a> + <psi,b> (3) and, with f_probe the potential one more u-update in the loop's
//           operand type gives (its ln S = ln a - f_probe / eps where a > 0), sum a |S_probe / S - 1|
//           (5: the row-marginal error that this update would make through its products alone).
//           Slot 4, the column-mass error, comes from k_colerr.
//   RO_CX, RO_CY: M = Scx or Scy, the transport cost's x or y part (slot 2 or 6).
//   RO_TY:  M = Sy; T_y = M scale, written over M.
// (T_x is needed at column 0 only, where the integration reads it: k_tx_column.)
enum ReadoutRole { RO_S = 0, RO_CX = 1, RO_CY = 2, RO_TY = 4 };
constexpr int READOUT_SLOTS = 7;
template <int ROLE>
__global__ __launch_bounds__(NTHREADS) void k_readout(
    double* M, const unsigned* colkey, const double* lnS_prev, const double* lna, const double* lnb,
    const double* f, const double* psi, const double* f_probe, int n, int np, double eps,
    double* part /*[READOUT_SLOTS][batch][blocks]*/) {
  __shared__ double red[4];
  const int bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  const int nblk = gridDim.x;
  double acc[4] = {0, 0, 0, 0};
  const double inv_eps = 1.0 / eps;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (size_t)n * n;
       idx += (size_t)nblk * blockDim.x) {
    const int j = (int)(idx / n), k = (int)(idx % n);
    const size_t o = bz * plane + (size_t)j * np + k;
    const size_t oa = (size_t)j * np + k;
    const double shift = key_to_shift(colkey[(size_t)bz * np + k]);
    const double scale = exp(shift - lnS_prev[o]);
    if constexpr (ROLE == RO_TY) {
      M[o] = M[o] * scale;
      continue;
    }
    const double la = lna[oa];
    if constexpr (ROLE == RO_CX || ROLE == RO_CY) {
      if (la > -INFINITY) acc[0] += exp(la) * scale * M[o];
      continue;
    }
    if constexpr (ROLE == RO_S) {
      if (la > -INFINITY) {
        const double a = exp(la);
        const double rm = a * M[o] * scale;
        acc[0] += fabs(rm - a);
        acc[1] += rm;
        acc[2] += a * f[o];
        if (f_probe) {
          // ln S(V_T) in FP64 against the operand type's value
          const double lnS64 = shift + log(M[o]);
          const double lnSq = la - f_probe[o] * inv_eps;
          const double d = lnSq - lnS64;
          // both -inf: no term; any other NaN (a non-finite probe) counts as the pixel's whole mass
          const bool none = lnSq == -INFINITY && lnS64 == -INFINITY;
          acc[3] += none ? 0.0 : (d == d) ? a * fabs(expm1(d)) : a;
        }
      }
      const double lb = lnb[o];
      if (lb > -INFINITY) acc[2] += exp(lb) * psi[o];
    }
  }
  if constexpr (ROLE == RO_TY) return;
  const int B = gridDim.y;
  constexpr int NQ = ROLE == RO_S ? 4 : 1;
  constexpr int slot_s[4] = {0, 1, 3, 5};
  for (int q = 0; q < NQ; ++q) {
    const int sl = ROLE == RO_S ? slot_s[q] : ROLE == RO_CX ? 2 : 6;
    const double s = block_sum(acc[q], red);
    if (threadIdx.x == 0) part[((size_t)sl * B + bz) * nblk + blockIdx.x] = s;
  }
}

// T_x at column 0 (Eq. 9): Sx[j][0] = sum_L Lambda(j - L) Bx[0][L] with the moment operand's row
// for k = 0, Bx[0][L] = X_L exp(m_L - m'_0 + Z[L][0]) (k_colexpT MODE 1 for that one column: Z =
// ln(A0 Lambda) with the row shifts m and column keys m' of its k_rowexp / EPI_LOGROW product), then
// scaled as T = Sx exp(m'_0 - ln S_prev).  Lambda from its FP64 Toeplitz table (element 0 of chunk
// d + n_p - 1 is the value at distance d).  One block per row j and target.
__global__ __launch_bounds__(NTHREADS) void k_tx_column(const double* Z, const double* mrow, const unsigned* colkey,
                                                        const double* lamT, const double* lnS_prev, int n, int np,
                                                        double* tcol) {
  __shared__ double red[4];
  const int j = blockIdx.x, bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  const double mk = key_to_shift(colkey[(size_t)bz * np]);
  const double xsc = 1.0 / sqrt((double)n);
  double s = 0.0;
  for (int L = threadIdx.x; L < n; L += blockDim.x) {
    const double zz = Z[bz * plane + (size_t)L * np];
    const double w = scaled_exp_op<double>((mrow[(size_t)bz * np + L] - mk) + zz, (double)(L - n / 2) * xsc);
    s += lamT[2 * (j - L + np - 1)] * w;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) tcol[(size_t)bz * np + j] = s * exp(mk - lnS_prev[bz * plane + (size_t)j * np]);
}

// Column-marginal L1 error of the returned plan (slot 4 of the read-out's partials): S' =
// Lambda u_T Lambda in FP64 arrives raw (divided by exp(m'_k), the column keys), so
// ln S' = m'_k + ln S'raw and the column mass is exp(psi/eps + ln S'); per-block sums over the
// pixels of |mass - b|, or of the mass where b = 0.  Same grid and summation order as k_readout.
__global__ __launch_bounds__(NTHREADS) void k_colerr(const double* S, const unsigned* colkey, const double* psi,
                                                      const double* lnb, int n, int np, double eps,
                                                      double* part /*[READOUT_SLOTS][batch][blocks]*/) {
  __shared__ double red[4];
  const int bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  const double inv_eps = 1.0 / eps;
  double acc = 0.0;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (size_t)n * n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / n), k = (int)(idx % n);
    const size_t o = bz * plane + (size_t)j * np + k;
    const double v = S[o];
    const double lnSp = (v > 0.0) ? key_to_shift(colkey[(size_t)bz * np + k]) + log(v) : -INFINITY;
    const double lb = lnb[o];
    const double cmass = exp(psi[o] * inv_eps + lnSp);
    acc += (lb > -INFINITY) ? fabs(cmass - exp(lb)) : cmass;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[((size_t)4 * gridDim.y + bz) * gridDim.x + blockIdx.x] = s;
}

// Deterministic final sums of the read-out partials: out[q][bz] for q < READOUT_SLOTS.
__global__ void k_sum_parts(const double* part, int nblk, double* out) {
  __shared__ double red[4];
  const int q = blockIdx.x, bz = blockIdx.y, B = gridDim.y;
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) v += part[((size_t)q * B + bz) * nblk + i];
  v = block_sum(v, red);
  if (threadIdx.x == 0) out[(size_t)q * B + bz] = v;
}

// Trapezoid integration (step 1/sqrt(n)): phi[j][0] from T_x's column 0 (txc[bz][j]) along j, then
// along k with Ty.  One block per row; rowpart[bz][j] = sum_k a_jk phi_jk for the a-weighted mean.
__global__ __launch_bounds__(NTHREADS) void k_integrate(const double* txc, const double* Ty, const double* lna,
                                                        int n, int np, double* phi, double* rowpart) {
  __shared__ double red[4];
  __shared__ double tsum[NTHREADS];
  const int j = blockIdx.x, bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  const double hh = 0.5 / sqrt((double)n);
  // phi[j][0] = sum_{i<j} h/2 (Tx[i][0] + Tx[i+1][0])
  double c = 0.0;
  for (int i = threadIdx.x; i < j; i += blockDim.x)
    c += hh * (txc[(size_t)bz * np + i] + txc[(size_t)bz * np + i + 1]);
  const double base = block_sum(c, red);
  // scan of increments d_k = h/2 (Ty[j][k-1] + Ty[j][k]) over contiguous chunks per thread
  const double* ty = Ty + bz * plane + (size_t)j * np;
  const int chunk = (n + NTHREADS - 1) / NTHREADS;
  const int k0 = threadIdx.x * chunk, k1 = min(n, k0 + chunk);
  double s = 0.0;
  for (int k = max(k0, 1); k < k1; ++k) s += hh * (ty[k - 1] + ty[k]);
  tsum[threadIdx.x] = s;
  __syncthreads();
  double prefix = 0.0;
  for (int t = 0; t < (int)threadIdx.x; ++t) prefix += tsum[t];
  double run = base + prefix;
  double wsum = 0.0;
  double* ph = phi + bz * plane + (size_t)j * np;
  const double* la = lna + (size_t)j * np;
  for (int k = k0; k < k1; ++k) {
    if (k >= 1) run += hh * (ty[k - 1] + ty[k]);
    ph[k] = run;
    if (la[k] > -INFINITY) wsum += exp(la[k]) * run;
  }
  wsum = block_sum(wsum, red);
  if (threadIdx.x == 0) rowpart[(size_t)bz * n + j] = wsum;
}

// Remove the a-weighted mean and write the caller's dense [batch][n][n] layout.
__global__ __launch_bounds__(NTHREADS) void k_center(const double* phi, const double* rowpart, int n, int np,
                                                     double* out) {
  __shared__ double red[4];
  const int j = blockIdx.x, bz = blockIdx.y;
  double v = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x) v += rowpart[(size_t)bz * n + r];
  const double mean = block_sum(v, red);
  const double* ph = phi + (size_t)bz * np * np + (size_t)j * np;
  double* o = out + ((size_t)bz * n + j) * n;
  for (int k = threadIdx.x; k < n; k += blockDim.x) o[k] = ph[k] - mean;
}

// ------------------------------------------------------------------ reverse mode
// acc += eps * v where the mask ln(marginal) > -inf holds (reverse of psi = eps ln b - ...).
__global__ void k_axpy_masked(const double* v, const double* lnm, int n, int np, double eps, double* acc) {
  const int bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (size_t)n * n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t o = bz * plane + (size_t)(idx / n) * np + (idx % n);
    if (lnm[o] > -INFINITY) acc[o] += eps * v[o];
  }
}

// out = dD[bz] * marginal (masked), in the padded layout; marginal = exp(lnm).
__global__ void k_seed(const double* dD, const double* lnm, long long sMarg, int n, int np, double* out) {
  const int bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < plane;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / np), k = (int)(idx % np);
    double v = 0.0;
    if (j < n && k < n) {
      const double l = lnm[bz * sMarg + idx];
      if (l > -INFINITY) v = dD[bz] * exp(l);
    }
    out[bz * plane + idx] = v;
  }
}

// Transpose of the trapezoid integration with the a-weighted mean removed.
// Step 1 (one block per row): row sums of dphi (caller layout) and of a * total later.
__global__ __launch_bounds__(NTHREADS) void k_rowsum_dense(const double* x, int n, double* rowsum) {
  __shared__ double red[4];
  const int j = blockIdx.x, bz = blockIdx.y;
  const double* r = x + ((size_t)bz * n + j) * n;
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) s += r[k];
  s = block_sum(s, red);
  if (threadIdx.x == 0) rowsum[(size_t)bz * n + j] = s;
}

// Step 2 (one block per row j): pb = dphi - a * total; Tby[j][m] = h/2 (R[m] + R[m-1]) with
// R[i] = sum_{k>i} pb[j][k]; cbar[j] = sum_k pb[j][k].
__global__ __launch_bounds__(NTHREADS) void k_int_adj_rows(const double* dphi, const double* rowsum,
                                                           const double* lna, int n, int np, double* Tby,
                                                           double* cbar, double* Tbx) {
  __shared__ double red[4];
  __shared__ double tsum[NTHREADS];
  const int j = blockIdx.x, bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  double t = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x) t += rowsum[(size_t)bz * n + r];
  const double total = block_sum(t, red);
  const double* dp = dphi + ((size_t)bz * n + j) * n;
  const double* la = lna + (size_t)j * np;
  const double hh = 0.5 / sqrt((double)n);
  for (int k = threadIdx.x; k < n; k += blockDim.x) Tbx[bz * plane + (size_t)j * np + k] = 0.0;
  // contiguous chunk per thread, scanned from the right
  const int chunk = (n + NTHREADS - 1) / NTHREADS;
  const int k0 = threadIdx.x * chunk, k1 = min(n, k0 + chunk);
  double s = 0.0;
  for (int k = k0; k < k1; ++k) s += dp[k] - (la[k] > -INFINITY ? exp(la[k]) : 0.0) * total;
  tsum[threadIdx.x] = s;
  __syncthreads();
  double suffix = 0.0;  // sum of pb over chunks to the right
  for (int q = threadIdx.x + 1; q < NTHREADS; ++q) suffix += tsum[q];
  double* ty = Tby + bz * plane + (size_t)j * np;
  // R[i] = suffix_after(i); walk i from k1-1 down to k0
  double run = suffix;  // sum_{k >= k1} pb
  for (int i = k1 - 1; i >= k0; --i) {
    const double Ri = run;  // sum_{k > i} pb
    const double Rim1 = run + (dp[i] - (la[i] > -INFINITY ? exp(la[i]) : 0.0) * total);  // R[i-1]
    double v = 0.0;
    if (i <= n - 2) v += hh * Ri;
    if (i >= 1) v += hh * Rim1;
    ty[i] = v;
    run = Rim1;
  }
  double rs = 0.0;
  for (int q = 0; q < NTHREADS; ++q) rs += tsum[q];
  if (threadIdx.x == 0) cbar[(size_t)bz * n + j] = rs;
}

// Step 3 (one block per target): Tbx[m][0] = h/2 (Rc[m] + Rc[m-1]) with Rc[i] = sum_{j>i} cbar[j];
// the other columns of Tbx were zeroed by step 2.
__global__ __launch_bounds__(NTHREADS) void k_int_adj_col(const double* cbar, int n, int np, double* Tbx) {
  const int bz = blockIdx.x;
  const size_t plane = (size_t)np * np;
  double* tx = Tbx + bz * plane;
  if (threadIdx.x == 0) {
    const double hh = 0.5 / sqrt((double)n);
    const double* cb = cbar + (size_t)bz * n;
    double run = 0.0;  // sum_{j > i} cbar
    for (int i = n - 1; i >= 0; --i) {
      const double Ri = run, Rim1 = run + cb[i];
      double v = 0.0;
      if (i <= n - 2) v += hh * Ri;
      if (i >= 1) v += hh * Rim1;
      tx[(size_t)i * np] = v;
      run = Rim1;
    }
  }
}

// w = Tbx * Tx + Tby * Ty (padded layout, valid pixels only).  Tbx, the adjoint of the integration,
// is nonzero only in column 0, where T_x is given as txc[bz][j].
__global__ void k_moment_weight(const double* Tbx, const double* txc, const double* Tby, const double* Ty, int n,
                                int np, double* w) {
  const int bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (size_t)n * n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / n), k = (int)(idx % n);
    const size_t o = bz * plane + (size_t)j * np + k;
    w[o] = (k == 0 ? Tbx[o] * txc[(size_t)bz * np + j] : 0.0) + Tby[o] * Ty[o];
  }
}

// Sums of the normalisation Jacobian, in fixed order: k_grad_rows forms per-row partials (one block
// per row and target) of sum lbbar and sum b psi over the pixels with b > 0; k_grad_sums adds a
// target's rows and writes out[bz] = sum lbbar, out[B + bz] = dD sum b psi.
__global__ __launch_bounds__(NTHREADS) void k_grad_rows(const double* lbbar, const double* psi, const double* lnb,
                                                        int n, int np, double* parts) {
  __shared__ double red[4];
  const int r = blockIdx.x, bz = blockIdx.y;
  const size_t o0 = (size_t)bz * np * np + (size_t)r * np;
  double s0 = 0.0, s1 = 0.0;
  for (int k = threadIdx.x; k < n; k += NTHREADS) {
    const double l = lnb[o0 + k];
    if (l > -INFINITY) {
      s0 += lbbar[o0 + k];
      s1 += exp(l) * psi[o0 + k];
    }
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    parts[((size_t)bz * 2) * n + r] = s0;
    parts[((size_t)bz * 2 + 1) * n + r] = s1;
  }
}

__global__ __launch_bounds__(NTHREADS) void k_grad_sums(const double* parts, const double* dD, int n, double* out) {
  __shared__ double red[4];
  const int bz = blockIdx.x, B = gridDim.x;
  double s0 = 0.0, s1 = 0.0;
  for (int r = threadIdx.x; r < n; r += NTHREADS) {
    s0 += parts[((size_t)bz * 2) * n + r];
    s1 += parts[((size_t)bz * 2 + 1) * n + r];
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    out[bz] = s0;
    out[B + bz] = dD[bz] * s1;
  }
}

// dL/dG = (2G/Z)(bbar - <bbar, b>), bbar = lbbar / b + dD psi (b = G^2/Z), written as
// 2 lbbar / G + (2G/Z)(dD psi - sum lbbar - dD <psi,b>); zero where G = 0.  G is rebuilt from
// the stored ln b and Z = sum G^2 of the solve: G = exp((ln b + ln Z)/2).
__global__ void k_grad_final(const double* rowsum_G, const double* lbbar, const double* psi, const double* lnb,
                             const double* dD, const double* sums, int n, int np, double* dG) {
  __shared__ double Zs;
  const int bz = blockIdx.y, B = gridDim.y;
  const size_t plane = (size_t)np * np;
  if (threadIdx.x == 0) {
    double z = 0.0;
    for (int r = 0; r < n; ++r) z += rowsum_G[(size_t)bz * n + r];
    Zs = z;
  }
  __syncthreads();
  const double Z = Zs, lz = log(Zs);
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (size_t)n * n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t o = bz * plane + (size_t)(idx / n) * np + (idx % n);
    double v = 0.0;
    if (lnb[o] > -INFINITY) {
      const double g = exp(0.5 * (lnb[o] + lz));
      v = 2.0 * lbbar[o] / g + (2.0 * g / Z) * (dD[bz] * psi[o] - sums[bz] - sums[B + bz]);
    }
    dG[(size_t)bz * n * n + idx] = v;
  }
}

__global__ void k_fill(double* x, size_t count, double value) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    x[i] = value;
}

}  // namespace fot
