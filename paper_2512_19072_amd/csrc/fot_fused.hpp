// Fused half-step of the FOT iteration for gfx950: two kernels per half-step.
//
// One half-step of Algorithm 1 (arXiv 2512.19072, Sec. 3, Eq. 7 or Eq. 8) computes, in the log
// domain, ln S = ln(Lambda . exp(P/eps) . Lambda) and the new potential eps (ln m - ln S).
// Every operand the per-axis GEMMs consume is stored normalised per 64-wide (or 32-wide) block of
// its K index by an integer power of two:
//
//   At[L][M] = exp(P_LM/eps - K[L][blk(M)] ln 2)      (pass-1 operand, max of a block in [1/2, 1])
//   Bt[k][L] = W[L][k] 2^{-K'[k][blk(L)]}              (pass-2 operand, transposed)
//
// The consuming GEMM runs each block through the MFMA in the operand precision and adds the
// block's FP32 (or FP64) partial sum into an FP64 accumulator scaled by the exact power of two
// 2^{K - max K}.  So no global row or column maximum is ever needed: each producer tile
// normalises its own blocks, the consumer rescales exactly, and neither atomics nor separate
// exponentiation kernels are left in the loop.
//
//   pass 1  W~ = At . Lambda^T, W = W~ 2^{R_L}; epilogue writes Bt (block exponents by frexp, no
//           transcendental) and the exponent table K'.
// At small eps Lambda itself spans more than the operand type's range; it is then stored the same
// way, Lambda[k][M] = Lambda~[k][M] 2^{KL[k][blk(M)]} (KL <= 0), and each block's partial sum is
// rescaled by the sum of both operands' exponents (the LN form of the kernels).  Raw Lambda is
// not staged with the K stages: it depends on i - k only, and its fragments are read from a
// Toeplitz table (one 16-byte chunk per starting distance; BF16x3: one table of the hi and one of
// the lo halves) that each workgroup copies into LDS once.
//   pass 2  S~ = Lambda . Bt^T, ln S = R'_k ln 2 + ln S~; epilogue updates the potential, the
//           marginal-error partial, and writes the next pass-1 operand At and its exponents.
#pragma once

#include <climits>
#include <type_traits>

#include "fot_kernels.hpp"

namespace fot {

constexpr int KSENT = -(1 << 30);          // exponent of an all-zero block
constexpr double KMIN = -1.0e9;            // lowest exponent of a block holding a finite value
constexpr double LN2 = 0.69314718055994530942;
constexpr double INV_LN2 = 1.44269504088896340736;
// ln 2 split so that e * LN2_HI is exact for |e| < 2^21 (head has 32 significant bits)
constexpr double LN2_HI = 6.93147180369123816490e-01;
constexpr double LN2_LO = 1.90821492927058770002e-10;

struct FusedArgs {
  const void* A;            // [batch][np][np] pass-1: At;  pass-2: Lambda (shared, sA = 0)
  const void* B;            // [batch][np][np] pass-1: Lambda (shared); pass-2: Bt
  long long sA, sB;
  int n, np, nk;
  int nbA;                  // exponent blocks per row of the pass-1 operand (np / BN)
  int nbT;                  // exponent blocks per row of the pass-2 operand (np / BM)
  int xcd_swizzle;
  const int* kexp;          // [batch][np][nb] exponents of the block-normalised operand (pass 1: A, pass 2: B)
  // pass 1 outputs
  void* outT;               // [batch][np][np] Bt for pass 2
  int* kexpT;               // [batch][np][nb]
  const double* pend_parts; // marginal-error partials of the previous update (nullptr: none)
  int pend_tiles;
  double* pend_out;         // [batch]
  // pass 2
  const double* lnmarg;     // ln a or ln b, [np][np] with batch stride sMarg
  long long sMarg;
  double* pot;              // potential updated in place
  double* lnS_out;          // optional copy of ln S
  double eps, inv_eps;
  double next_inv_eps;      // > 0: also write the next pass-1 operand with this 1/eps
  void* nextA;              // [batch][np][np]
  int* kexpN;               // [batch][np][nb]
  double* partials;         // [batch][tiles]
  int* flag;
  int err_on;               // pass 2: evaluate the marginal-error partial (reads the old potential)
  int band;                 // Lambda[i][k] is zero in the operand type for |i - k| > band (>= n: no zeros)
  const int* kexpL;         // LN form: [np][nb] exponents of the block-normalised Lambda (nb as kexp)
  int* range_slots;         // [batch][range_spt][2] or nullptr: per wave of a launch, the lowest range
                            // margin of its outputs (see range_margin) and the lowest `iter` at which
                            // one fell below range_thr (one slot per wave: no two waves share an address)
  int range_spt;            // slots per target
  int iter;                 // iteration index recorded by the range check
  int range_thr;            // an output whose margin is below this fails the range check
  // pass 2 of a reverse half-step (k_fused<..., ADJ = true>): pot is read only (the potential P of
  // the update being differentiated), lnmarg masks the output
  double* adj_out;          // [batch][np][np] updated output
  double adj_scale;         // weight w of every term
  int adj_coords;           // bit 0: w also times the row coordinate (i - n/2)/sqrt n; bit 1: column
  int adj_acc;              // add to adj_out instead of overwriting it
  double* adj_lb;           // or nullptr: also adj_lb += adj_lb_scale * (new adj_out), masked alike
  double adj_lb_scale;
  const double* adj_next_L; // or nullptr: write the pass-1 operand of the next reverse half-step,
                            // v = the new output with this L (as k_adj_prep), to nextA / kexpN,
                            // instead of adj_out (which then only the next operand needs)
};

// Range check of a contraction output.  Each term of a block's partial sum is a product of two
// factors that are at most 1 after the block normalisation; a term the operand type cannot hold
// (a factor or the product below the type's smallest normal number, flushed or rounded) is off by
// less than 2^-125 (FP32, BF16, BF16x3), 2^-1021 (FP64) or 2^-23 (FP16) of its block's scale.  An
// output formed from n terms therefore loses less than n 2^-125 (...) of the largest block scale
// it was formed from.  Its margin is the binary exponent of the output relative to that scale
// (frexp, so an output of 2^e x [1/2, 1) with scale 2^s has margin e - s; an output of zero
// from a line with mass has margin RANGE_ZERO): the relative loss is below n 2^-125 2^-margin.
// Each wave records the lowest margin of its outputs, and the iteration at which a margin first fell
// below a threshold the host derives from the type, in a slot of its own; the host reduces them.
constexpr int RANGE_ZERO = -100000;
__device__ __forceinline__ int range_margin(double v, int scale) {
  int ex;
  (void)frexp(v, &ex);
  return v > 0.0 ? ex - scale : RANGE_ZERO;
}

// minimum over the 64 lanes of a wave: rows of 16 by DPP, then the four row results by readlane
// (no LDS traffic); every lane returns it
__device__ __forceinline__ int wave_min_int(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));   // row_half_mirror
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));   // row_mirror
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// exp(x - K ln 2) rounded to the operand type, with the K of a block's maximum.  The prep
// kernel and the pass-2 epilogue both use these two functions, so the operand built after a
// replay from a checkpoint is bit-identical to the one built inside the iteration.
// block_exponent is monotone in x, so the exponent of a block's maximum equals the maximum of
// its elements' exponents: the pass-2 epilogue reduces integers, the prep kernel doubles.
__device__ __forceinline__ int block_exponent(double xmax) {
  return (xmax > -INFINITY) ? (int)ceil(fmax(xmax * INV_LN2, KMIN)) : KSENT;
}
// 2^y by the hardware exponential (V_EXP_F32, about 1 ulp) of y rounded to FP32.
__device__ __forceinline__ float exp2_hw(double y) { return __builtin_amdgcn_exp2f((float)y); }

// exp(x - K ln 2) = 2^(x / ln 2 - K): the exponent is formed in FP64 (x reaches 1e4 in
// magnitude) and lies in (-1, 0] for a block's largest element, so its FP32 rounding costs less
// than one ulp of the result there; elements far below the block maximum, whose exponent is
// rounded more coarsely or underflows, are negligible in every sum they enter.
template <typename T>
__device__ __forceinline__ T block_operand(double x, int K) {
  if constexpr (sizeof(T) == 8)
    // (an explicit FMA: the compiler may contract x - K ln2 differently where the function is
    // inlined, and the prep kernel and the pass-2 epilogue must produce the same bits)
    return (K == KSENT) ? 0.0 : exp(fma(-(double)K, LN2, x));
  else
    return (K == KSENT) ? T{} : from_float<T>(exp2_hw(fma(x, INV_LN2, -(double)K)));
}

// exp(x) and exp(d) - 1 (d < 10) in FP32 for the marginal-error terms, which need a few
// significant digits: the argument is rounded to FP32 first (|x| stays below a few hundred where
// the result is not negligible, so that costs under 1e-5 relative), then a short series below
// |d| = 0.03 and the hardware exponential otherwise.
constexpr float INV_LN2F = 1.44269504088896340736f;
__device__ __forceinline__ float exp_err(float x) { return __builtin_amdgcn_exp2f(x * INV_LN2F); }
__device__ __forceinline__ float expm1_err(float d) {
  const float series = d * (1.0f + d * (0.5f + d * (1.0f / 6.0f + d * (1.0f / 24.0f))));
  const float direct = exp_err(d) - 1.0f;
  return fabsf(d) < 0.03f ? series : direct;
}

// ln v of an FP32-accumulated contraction: v = m 2^e exactly (frexp, m in [1/2, 1)), then
// log2 m by the hardware logarithm (V_LOG_F32) of m rounded to FP32.  The absolute error is about
// 1e-7, the size of the relative rounding error that FP32 operands leave in v itself.  Zero,
// infinity and NaN map to -inf, +inf and NaN.
__device__ __forceinline__ double log_op32(double v) {
  int e;
  const double m = frexp(v, &e);
  return ((double)e + (double)__builtin_amdgcn_logf((float)m)) * LN2;
}

// max over the 16 lanes of each row of a wave (DPP: quad swaps, then half-row and row mirrors)
__device__ __forceinline__ int row16_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));  // row_mirror
  return v;
}

// Natural logarithm in FP64 (within a few ulp) for the log-domain update: v = m 2^e with m in
// [1/sqrt 2, sqrt 2), ln m = 2 atanh(s) with s = (m - 1)/(m + 1), |s| < 0.172, summed by its odd
// power series to s^19 (truncation below 2^-55 relative), plus e ln 2 in two parts.  Zero,
// infinity and NaN take the library path.
__device__ __forceinline__ double log_fp64(double v) {
  if (!(v > 0.0 && v < INFINITY)) return log(v);
  int e;
  double m = frexp(v, &e);
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    --e;
  }
  const double num = m - 1.0, den = m + 1.0;  // num is exact
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  double q = num * r;
  q = fma(fma(-q, den, num), r, q);
  const double s2 = q * q;
  double t = 1.0 / 19.0;
  t = fma(t, s2, 1.0 / 17.0);
  t = fma(t, s2, 1.0 / 15.0);
  t = fma(t, s2, 1.0 / 13.0);
  t = fma(t, s2, 1.0 / 11.0);
  t = fma(t, s2, 1.0 / 9.0);
  t = fma(t, s2, 1.0 / 7.0);
  t = fma(t, s2, 1.0 / 5.0);
  t = fma(t, s2, 1.0 / 3.0);
  const double q2 = 2.0 * q;
  const double lnm = fma(q2 * s2, t, q2);
  const double de = (double)e;
  return fma(de, LN2_HI, fma(de, LN2_LO, lnm));
}

// m e^x 2^e2 in FP64 without forming e^x alone, which can overflow or underflow where the product
// does not (m and x finite): x = k ln 2 + r by Cody-Waite reduction (ln 2 split into a head of 32
// significant bits, so that k ln2_hi is exact for |k| < 2^21, and a tail), |r| <= ln2 / 2; e^r by
// its Taylor series through r^13 / 13! (the next term is below 5e-18 of the sum); then
// ldexp(m e^r, k + e2).  Within a few ulp.
__device__ __forceinline__ double mul_exp_fp64(double m, double x, int e2) {
  constexpr double LN2_HI = 0x1.62e42feep-1, LN2_LO = 0x1.a39ef35793c76p-33;
  const double k = fmin(fmax(rint(x * INV_LN2), -4000.0), 4000.0);
  const double r = fma(-k, LN2_LO, fma(-k, LN2_HI, x));
  double t = 1.6059043836821613e-10;             // 1/13!
  t = fma(t, r, 2.08767569878681e-09);           // 1/12!
  t = fma(t, r, 2.505210838544172e-08);
  t = fma(t, r, 2.755731922398589e-07);
  t = fma(t, r, 2.7557319223985893e-06);
  t = fma(t, r, 2.48015873015873e-05);
  t = fma(t, r, 1.984126984126984e-04);
  t = fma(t, r, 1.388888888888889e-03);
  t = fma(t, r, 8.333333333333333e-03);
  t = fma(t, r, 4.1666666666666664e-02);
  t = fma(t, r, 1.6666666666666666e-01);
  t = fma(t, r, 0.5);
  t = fma(t, r, 1.0);
  t = fma(t, r, 1.0);
  const int ex = (int)k + max(min(e2, 4000), -4000);
  return ldexp(m * t, ex);
}

// m e^x 2^e2 as accurate as an FP32-accumulated contraction (about 1e-7 relative): x / ln 2 in
// FP64 split into its integer part k and fraction f, 2^f by the hardware exponential (V_EXP_F32)
// of f rounded to FP32, then ldexp(m 2^f, k + e2).
__device__ __forceinline__ double mul_exp_op32(double m, double x, int e2) {
  const double y = x * INV_LN2;
  const double k = fmin(fmax(floor(y), -4000.0), 4000.0);
  const double t = (double)__builtin_amdgcn_exp2f((float)(y - k));
  return ldexp(m * t, (int)k + max(min(e2, 4000), -4000));
}

// 64-bit DPP move (two 32-bit halves), CTRL a DPP16 row control
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = (int)b, hi = (int)(b >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)h2 << 32) | (unsigned)l2);
}

// Sum over the 64 lanes of a wave in a fixed order: rows of 16 by DPP, then the four row sums
// in row order.  Every lane returns the same value.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  const long long b = __double_as_longlong(v);
  const int lo = (int)b, hi = (int)(b >> 32);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int l = __builtin_amdgcn_readlane(lo, 16 * r), h = __builtin_amdgcn_readlane(hi, 16 * r);
    s += __longlong_as_double(((long long)h << 32) | (unsigned)l);
  }
  return s;
}

// max over groups of XB consecutive lanes (XB = 32 or 64; every lane of the wave active): rows of
// 16 lanes by DPP (as wave_min_int), then the rows of the group by readlane (no LDS traffic)
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int XB>
__device__ __forceinline__ double group_max(double v) {
  static_assert(XB == 32 || XB == 64, "groups of 32 or 64 lanes");
  v = fmax(v, dpp_f64<0xB1>(v));    // quad_perm [1,0,3,2]
  v = fmax(v, dpp_f64<0x4E>(v));    // quad_perm [2,3,0,1]
  v = fmax(v, dpp_f64<0x141>(v));   // row_half_mirror
  v = fmax(v, dpp_f64<0x140>(v));   // row_mirror
  const double r01 = fmax(readlane_f64(v, 0), readlane_f64(v, 16));
  const double r23 = fmax(readlane_f64(v, 32), readlane_f64(v, 48));
  if constexpr (XB == 64) return fmax(r01, r23);
  return (threadIdx.x & 63) < 32 ? r01 : r23;
}

// Block-normalised pass-1 operand of a potential P (FP64 [batch][np][np]), blocks of XB columns.
// Launched on (np^2 / 1024, batch) workgroups of 256: a workgroup covers PREP_U consecutive runs of
// 256 elements, one element of each per thread.  The loads are unconditional (the padded plane is
// allocated; padding values are discarded by a select) and all issued before any use: a load under
// a branch is awaited inside the branch, which serialises them.  np is a multiple of 64, so a wave
// holds 64 consecutive columns of one row and whole blocks.
constexpr int PREP_U = 4;
template <typename T, int XB>
__global__ __launch_bounds__(256) void k_prep_blocks(const double* P, int n, int np, double inv_eps, T* out,
                                                     int* kexp) {
  const int bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  double x[PREP_U];
#pragma unroll
  for (int u = 0; u < PREP_U; ++u) {
    const unsigned idx = (blockIdx.x * PREP_U + u) * 256u + threadIdx.x;   // < np^2 <= 2^26
    x[u] = P[bz * plane + idx];
  }
#pragma unroll
  for (int u = 0; u < PREP_U; ++u) {
    const unsigned idx = (blockIdx.x * PREP_U + u) * 256u + threadIdx.x;
    const int j = (int)(idx / (unsigned)np), k = (int)(idx - (unsigned)j * (unsigned)np);
    x[u] = (j < n && k < n) ? x[u] * inv_eps : -INFINITY;
  }
#pragma unroll
  for (int u = 0; u < PREP_U; ++u) {
    const unsigned idx = (blockIdx.x * PREP_U + u) * 256u + threadIdx.x;   // < np^2 <= 2^26
    const int j = (int)(idx / (unsigned)np), k = (int)(idx - (unsigned)j * (unsigned)np);
    const int K = block_exponent(group_max<XB>(x[u]));
    store_op<T>(out + bz * plane + (size_t)j * np, k, x[u] > -INFINITY ? block_operand<T>(x[u], K) : T{});
    if (k % XB == 0) kexp[((size_t)bz * np + j) * (np / XB) + k / XB] = K;
  }
}

// Signed block-normalised pass-1 operand of a reverse half-step: w = v e^{-L} (v an adjoint, L a
// ln S of the forward iteration) as sign(v) exp(h - K ln 2) with h = ln|v| - L, K the exponent of
// its block's largest h (formed in the log domain: e^{-L} alone can overflow).  Launched like
// k_prep_blocks.
template <typename T, int XB>
__global__ __launch_bounds__(256) void k_adj_prep(const double* v, const double* L, int n, int np, T* out,
                                                  int* kexp) {
  const int bz = blockIdx.y;
  const size_t plane = (size_t)np * np;
  double vv[PREP_U], lv[PREP_U];
#pragma unroll
  for (int u = 0; u < PREP_U; ++u) {
    const unsigned idx = (blockIdx.x * PREP_U + u) * 256u + threadIdx.x;   // < np^2 <= 2^26
    vv[u] = v[bz * plane + idx];
    lv[u] = L[bz * plane + idx];
  }
#pragma unroll
  for (int u = 0; u < PREP_U; ++u) {
    const unsigned idx = (blockIdx.x * PREP_U + u) * 256u + threadIdx.x;
    const int j = (int)(idx / (unsigned)np), k = (int)(idx - (unsigned)j * (unsigned)np);
    if (!(j < n && k < n)) vv[u] = 0.0;
  }
#pragma unroll
  for (int u = 0; u < PREP_U; ++u) {
    const unsigned idx = (blockIdx.x * PREP_U + u) * 256u + threadIdx.x;   // < np^2 <= 2^26
    const int j = (int)(idx / (unsigned)np), k = (int)(idx - (unsigned)j * (unsigned)np);
    // (the logarithm as accurate as the operand type needs: FP64 for FP64 operands)
    const double lg = (sizeof(T) == 8) ? log_fp64(fabs(vv[u])) : log_op32(fabs(vv[u]));
    const double h = (vv[u] != 0.0) ? lg - lv[u] : -INFINITY;
    const int K = block_exponent(group_max<XB>(h));
    const T x = block_operand<T>(h, K);
    store_op<T>(out + bz * plane + (size_t)j * np, k, vv[u] < 0.0 ? (T)(-x) : x);
    if (k % XB == 0) kexp[((size_t)bz * np + j) * (np / XB) + k / XB] = K;
  }
}

// Block-normalised Lambda (LN form): row i holds Lambda[i][k] = exp(-(i - k)^2 / (2 n^2 eps)) as
// Lambda~ 2^{K} per block of XB columns, K the exponent of the block's largest entry; one wave per
// row.  Rows and columns beyond n hold the same formula (the operands they meet there are zero).
template <typename T, int XB>
__global__ __launch_bounds__(64) void k_lambda_blocks(int n, int np, double inv_eps, T* out, int* kexp) {
  const int i = blockIdx.x, lane = threadIdx.x;
  const int nb = np / XB;
  const double c = inv_eps / (2.0 * (double)n * (double)n);
  T* o = out + (size_t)i * np;
  int* ko = kexp + (size_t)i * nb;
  for (int c0 = 0; c0 < np; c0 += 64) {
    const int k = c0 + lane;
    const double d = (double)(i - k);
    const double x = -(d * d) * c;
    const int K = block_exponent(group_max<XB>(x));
    store_op<T>(o, k, block_operand<T>(x, K));
    if (lane % XB == 0) ko[k / XB] = K;
  }
}

// Wait until at most N vector-memory loads of this wave are outstanding (direct LDS loads
// included: they complete in issue order with the others).
template <int N>
__device__ __forceinline__ void vm_wait() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (0x7 << 4) | (0xF << 8) | ((N >> 4) << 14));
}

// Workgroup barrier that publishes LDS writes only: it waits for this wave's LDS operations
// (lgkmcnt) but not for its global stores, which __syncthreads' release fence would also wait for
// (in an epilogue that had just stored the potential, that wait was the store latency).  The
// compiler-only fences keep LDS accesses on their side of it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xF | (0x7 << 4) | (0x0 << 8) | (0x3 << 14));   // lgkmcnt(0)
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// 16-byte global -> LDS load of this lane's source; the wave's 64 lanes fill the 1 KB at
// lds_dst (wave-uniform) in lane order.  Written in assembly so that the compiler does not track
// it: its wait insertion would otherwise assume the load may overwrite LDS that fragment reads in
// flight still use and wait for all of them before every such load (measured: twice the time per
// launch).  Completion is awaited explicitly (vm_wait) before the workgroup barrier that
// publishes the stage, so the next stage stays in flight while the current one is read.  M0 (the
// LDS base of the load) is saved and restored inside the block, so the compiler's own use of M0
// is undisturbed and nothing reserved is clobbered; the load writes no VGPR.
__device__ __forceinline__ void dma16(const void* src, const unsigned char* lds_dst) {
  const unsigned lds_addr =
      __builtin_amdgcn_readfirstlane((unsigned)(size_t)(const __attribute__((address_space(3))) unsigned char*)lds_dst);
  unsigned saved;
  asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off\n\ts_mov_b32 m0, %0"
               : "=&s"(saved)
               : "v"(src), "s"(lds_addr)
               : "memory");
}

constexpr int FRAG_AHEAD = 2;  // LDS fragment reads issued this many MMA steps ahead
// Stage geometry (measured at 1024^2): 512-byte rows with two stages resident beat 256-byte rows
// with four (FP32 K loop 20.1 against 21.9 us, BF16 4.7 against 5.6 us): each stage ends in a
// workgroup barrier, after which the matrix cores idle until the next fragments arrive, and that
// cost per stage outweighs the deeper prefetch.
constexpr int FROWB = 512;      // bytes of one operand row per K stage of the fused kernels
constexpr int FUSED_NBUF = 2;   // K stages resident in LDS (one in flight while one is consumed)

// Toeplitz form of Lambda's operand (TZ): Lambda[i][k] depends on i - k only, so a tile's Lambda
// fragments are read from one table per workgroup instead of being staged with every K stage,
// which halves the bytes each workgroup fetches per stage.  Chunk c of the table is the 16 bytes
// of the 16 / sizeof(T) consecutive values Lambda(d), d = c - (n_p - 1) ... (one chunk for every
// starting distance, so that any fragment is one aligned 16-byte read, and the 16 rows of a
// fragment read 16 consecutive chunks: no bank conflicts).  The full table (2 n_p chunks, entries
// with |d| >= n_p zero) sits in device memory right after the n_p x n_p Lambda plane it is formed
// from (k_lam_chunks); a workgroup copies the window of at most n_p + LR chunks its tile uses
// (LR: its Lambda rows) into LDS, in 1 KB units.  BF16x3 operands (hi/lo layout) have two tables,
// of the hi and of the lo halves (8 halves per chunk), the lo one right after the hi one, and a
// workgroup copies a window of each.
__host__ __device__ inline size_t toeplitz_chunks_bytes(int np, bool paired = false) {
  return (size_t)(paired ? 64 : 32) * (size_t)np;
}
__host__ __device__ inline size_t toeplitz_table_bytes(int np, int lam_rows) {
  return ((size_t)16 * (size_t)(np + lam_rows) + 1023) / 1024 * 1024;
}

// The Toeplitz chunks of a Lambda plane (row 0 holds Lambda(|d|) for every d: all rows are the same
// function of i - k, padding included), written after the plane; one thread per chunk.
template <typename T>
__global__ void k_lam_chunks(T* lam, int np) {
  if constexpr (Mma<T>::PAIRED) {
    // hi/lo layout: value k of a row is half 2 (k & ~31) + (k & 31) (hi) and that + 32 (lo)
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= 2 * np) return;
    const unsigned short* row = (const unsigned short*)lam;
    unsigned short hv[8], lv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int d = abs(c - (np - 1) + e);
      const int h = 2 * (d & ~31) + (d & 31);
      hv[e] = d < np ? row[h] : (unsigned short)0;
      lv[e] = d < np ? row[h + 32] : (unsigned short)0;
    }
    u32x4 wh, wl;
    __builtin_memcpy(&wh, hv, 16);
    __builtin_memcpy(&wl, lv, 16);
    u32x4* t = (u32x4*)((unsigned char*)lam + (size_t)np * np * sizeof(T));
    t[c] = wh;
    t[2 * np + c] = wl;
    return;
  }
  typedef typename std::conditional<
      sizeof(T) == 2, unsigned short,
      typename std::conditional<sizeof(T) == 4, unsigned, unsigned long long>::type>::type EB;
  constexpr int EPC = 16 / (int)sizeof(T);
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 2 * np) return;
  const EB* row = (const EB*)lam;
  EB v[EPC];
#pragma unroll
  for (int e = 0; e < EPC; ++e) {
    const int d = abs(c - (np - 1) + e);
    v[e] = d < np ? row[d] : (EB)0;
  }
  u32x4 w;
  __builtin_memcpy(&w, v, 16);
  ((u32x4*)((unsigned char*)lam + (size_t)np * np * sizeof(T)))[c] = w;
}

// Launch with dynamic LDS of fused_dyn_lds<PASS, C, LN, TZ, PAIRED>(np) bytes (the exponent-
// difference table, in the LN form Lambda's exponent table for the tile's Lambda rows, and in the TZ
// form the window of Lambda's Toeplitz table, 16-byte aligned; BF16x3: the hi and the lo window).
template <int PASS, typename C>
constexpr int fused_scaled_rows() { return PASS == 1 ? C::BM : C::BN; }
template <int PASS, typename C, bool LN = false, bool TZ = false, bool PAIRED = false>
inline size_t fused_dyn_lds(int np) {
  const int xb = (PASS == 1 ? C::BN : C::BM) / C::XS;
  const int lam_rows = PASS == 1 ? C::BN : C::BM;
  size_t bytes = (size_t)(np / xb) * (fused_scaled_rows<PASS, C>() + (LN ? lam_rows : 0)) * sizeof(short);
  if (TZ) bytes = (bytes + 15) / 16 * 16 + (PAIRED ? 2 : 1) * toeplitz_table_bytes(np, lam_rows);
  return bytes;
}

// ADJ: the contraction of a reverse half-step (signed operands; pass 2 ends in the reverse update
// instead of the potential update).  TZ: Lambda's operand from the Toeplitz table (raw Lambda
// only; the LN form's block-normalised Lambda is not Toeplitz).
template <typename T, int PASS, typename C, int NBUF = FUSED_NBUF, bool LN = false, bool ADJ = false,
          bool TZ = false>
__global__ __launch_bounds__(C::THREADS) void k_fused(const FusedArgs p) {
  static_assert(NBUF >= 2, "at least double buffering");
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int BM = C::BM, BN = C::BN, RB = C::RB, CB = C::CB;
  constexpr int XB = (PASS == 1 ? BN : BM) / C::XS;   // K extent of one exponent block of this pass
  // exponent blocks of the outputs: pass 1's (the pass-2 operand's) span XB1 rows, the next
  // operand's (pass 2) XB2 columns; WPB1 / WPB2 waves along M / N share one
  constexpr int XB1 = BM / C::XS, XB2 = BN / C::XS;
  constexpr int WPB1 = XB1 / C::WTM, WPB2 = XB2 / C::WTN;
  static_assert(XB1 % C::WTM == 0 && XB2 % C::WTN == 0, "an exponent block holds whole wave tiles");
  constexpr int SR = fused_scaled_rows<PASS, C>(); // rows whose exponents scale the sums
  constexpr int HPS = FROWB / 64;                 // fragment steps per K stage
  constexpr int EPH = 64 / (int)sizeof(T);        // K elements per fragment step (4 lane groups;
                                                  // BF16x3: 32 values over a hi and a lo step)
  constexpr int HB = XB / EPH;                    // fragment steps per exponent block
  constexpr bool PAIRED = Mma<T>::PAIRED;
  // operand outputs (pass 1's Bt, pass 2's next At) as non-temporal stores for FP32 and FP64
  // operands: less to write back when the launch ends (measured: FP32 solves 2.5% and FP64 ones
  // 3% faster; the 16-bit kernels, which re-read their smaller operands sooner than they would
  // drain, 3% slower)
  constexpr bool NT_OPS = std::is_same<T, float>::value || std::is_same<T, double>::value;
  static_assert(HB >= 1 && XB % EPH == 0, "exponent blocks must hold whole fragment steps");
  static_assert(!PAIRED || (HB % 2 == 0 && HPS % 2 == 0), "hi/lo step pairs within a block and a stage");
  static_assert(!TZ || !LN, "the Toeplitz table holds raw Lambda");
  // rows staged per K stage: both operands, or (TZ) only the operand that is not Lambda
  constexpr int SROWS = TZ ? (PASS == 1 ? BM : BN) : BM + BN;
  // K-stage buffers as distinct objects, so that the compiler can tell a direct load into one
  // buffer from reads of another (it would otherwise wait for every load in flight)
  __shared__ __attribute__((aligned(1024))) unsigned char lds0[SROWS * FROWB];
  __shared__ __attribute__((aligned(1024))) unsigned char lds1[SROWS * FROWB];
  __shared__ __attribute__((aligned(1024))) unsigned char lds2[(NBUF > 2 ? SROWS : 1) * FROWB];
  __shared__ __attribute__((aligned(1024))) unsigned char lds3[(NBUF > 3 ? SROWS : 1) * FROWB];
  static_assert(NBUF <= 4, "four stage buffers at most");
  auto bufp = [](int j) -> unsigned char* { return j == 0 ? lds0 : j == 1 ? lds1 : j == 2 ? lds2 : lds3; };
  extern __shared__ __attribute__((aligned(16))) short dtab[];   // [np / XB][SR]: exponent - row reference
  constexpr int LR = PASS == 1 ? BN : BM;         // Lambda rows of the tile (output columns / rows)
  __shared__ int rref[SR];                        // reference exponent of each scaled row
  __shared__ double red[C::NW];
  // pass 2: row exponents of the next operand, [row][wave column] so that a row's entries are
  // one vector read
  __shared__ __attribute__((aligned(16))) int kred[BM][C::WGN];
  __shared__ __attribute__((aligned(16))) int ered[BN][C::WGM];   // pass 1: column exponent maxima, [column][wave row]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / C::WGN, wn = wave % C::WGN;
  const int r16 = lane & 15, g = lane >> 4;
  const int bz = blockIdx.z;
  const int n = p.n, np = p.np;
  const int nbk = PASS == 1 ? p.nbA : p.nbT;     // exponent blocks along this pass's K
  int tr, tc;
  tile_of(gridDim.x, gridDim.y, p.xcd_swizzle, &tr, &tc);
  const int row0 = tr * BM, col0 = tc * BN;
  const size_t plane = (size_t)np * np;
  // K stages [k_lo, k_lo + nks) whose Lambda block can be nonzero for this tile: Lambda is the
  // B operand of pass 1 (its rows are the output columns) and the A operand of pass 2 (rows =
  // output rows), and its entries vanish in the operand type beyond the band.  The skipped
  // stages would only add exact zeros, so the result is the same as with all stages (LN form: the
  // band is FP64's, and a skipped block would add at most 2^-1070 of its row's reference).
  constexpr int KPS = FROWB / (int)sizeof(T);      // K values per stage
  constexpr int SPB = XB > KPS ? XB / KPS : 1;     // stages per exponent block (FP64 operands: 2)
  int k_lo = 0, nks = p.nk;
  if (p.band < n) {
    const int lam0 = PASS == 1 ? col0 : row0, lamL = PASS == 1 ? BN : BM;
    const int lo = max(0, lam0 - p.band), hi = lam0 + lamL - 1 + p.band;
    k_lo = (lo / KPS) / SPB * SPB;   // the loop starts on an exponent block's first stage
    nks = min(p.nk, hi / KPS + 1) - k_lo;
  }

  // ---- operand staging: each K stage of the tile (BM rows of A, then BN rows of B, FROWB bytes
  // per row; TZ: only the rows of the operand that is not Lambda) is copied global -> LDS by
  // 16-byte direct loads (no register round trip).  A wave instruction fills 1 KB of LDS, lane l
  // at byte 16 l: 1024 / FROWB whole rows.  LDS rows are unpadded; the 16-byte chunk c of row r
  // sits in slot c ^ (r mod 16), so the fragment reads (16 rows, one chunk) hit 16 distinct
  // slots, i.e. all banks once.
  const size_t pitch = (size_t)np * sizeof(T);
  const unsigned char* Ab = (const unsigned char*)p.A + ((size_t)bz * p.sA) * sizeof(T) + (size_t)row0 * pitch;
  const unsigned char* Bb = (const unsigned char*)p.B + ((size_t)bz * p.sB) * sizeof(T) + (size_t)col0 * pitch;
  constexpr int RPU = 1024 / FROWB;                // rows per 1 KB load unit
  constexpr int CPR = FROWB / 16;                 // 16-byte chunks per row
  constexpr int UNITS = SROWS / RPU;              // 1 KB load units per stage
  constexpr int UPW = UNITS / C::NW;              // units per wave
  static_assert(UNITS % C::NW == 0 && BM % RPU == 0, "stage staging: whole units per wave, A/B split on a unit");
  const unsigned char* dsrc[UPW];
#pragma unroll
  for (int i = 0; i < UPW; ++i) {
    const int u = wave + C::NW * i;
    const int r = RPU * u + lane / CPR;
    const int c = (lane % CPR) ^ (r & 15);
    if constexpr (TZ)
      dsrc[i] = (PASS == 1 ? Ab : Bb) + (size_t)r * pitch + c * 16;
    else
      dsrc[i] = (r < BM ? Ab + (size_t)r * pitch : Bb + (size_t)(r - BM) * pitch) + c * 16;
  }
  auto stage_load = [&](int kk, unsigned char* dst) {
#pragma unroll
    for (int i = 0; i < UPW; ++i) dma16(dsrc[i] + (size_t)(kk + k_lo) * FROWB, dst + (wave + C::NW * i) * 1024);
  };

  // ---- prologue: stage 0 and the exponent table first (the table build waits for its loads,
  // and with them for stage 0), then the later stages and the epilogue inputs
  stage_load(0, bufp(0));

  // TZ: the window of Lambda's Toeplitz chunks this tile uses, copied into LDS (16-byte aligned
  // after the exponent table) like a stage.  The tile's Lambda rows are lam0 + lr (lr < LR) and its
  // K range starts at k_lo KPS, so the distances K - (lam0 + lr) start at d_lo = k_lo KPS - lam0 -
  // (LR - 1): the fragment of Lambda row lam0 + lr at K chunk c (K = c EPC ...) is window chunk
  // x = c EPC - k_lo KPS + LR - 1 - lr, the window has nch chunks, and every |d| is below n_p.
  // (BF16x3: a chunk holds 8 hi or 8 lo halves, and the lo window follows the hi one at tzlo)
  constexpr int EPC = PAIRED ? 8 : 16 / (int)sizeof(T);   // operand elements per 16-byte chunk
  unsigned char* const tzt = (unsigned char*)dtab + ((size_t)nbk * SR * sizeof(short) + 15) / 16 * 16;
  const int tzlo = PAIRED ? (int)toeplitz_table_bytes(np, LR) : 0;
  if constexpr (TZ) {
    const int lam0 = PASS == 1 ? col0 : row0;
    const int cbase = k_lo * KPS - lam0 - (LR - 1) + (np - 1);   // first chunk of the window (>= 0)
    const int nch = nks * KPS + LR - EPC;
    const u32x4* chunks = (const u32x4*)((const unsigned char*)(PASS == 1 ? p.B : p.A) + plane * sizeof(T));
    for (int u = wave; u * 64 < nch; u += C::NW)   // (lanes past the window copy its last chunk again)
      dma16(chunks + min(cbase + u * 64 + lane, 2 * np - 1), tzt + u * 1024);
    if constexpr (PAIRED)
      for (int u = wave; u * 64 < nch; u += C::NW)
        dma16(chunks + 2 * np + min(cbase + u * 64 + lane, 2 * np - 1), tzt + tzlo + u * 1024);
  }

  // exponent table of the block-normalised operand for this tile's scaled rows
  // (pass 1: A rows = output rows; pass 2: B rows = output columns)
  {
    const int srow0 = (PASS == 1) ? row0 : col0;
    const int* kx = p.kexp + ((size_t)bz * np + srow0) * nbk;
    for (int r = tid / 8; r < SR; r += C::THREADS / 8) {
      const int sub = tid % 8;
      int m = KSENT;
      for (int b = sub; b < nbk; b += 8) m = max(m, kx[(size_t)r * nbk + b]);
      m = max(m, __shfl_xor(m, 1, 64));
      m = max(m, __shfl_xor(m, 2, 64));
      m = max(m, __shfl_xor(m, 4, 64));
      if (sub == 0) rref[r] = m;
      for (int b = sub; b < nbk; b += 8) {
        const int d = kx[(size_t)r * nbk + b] - m;
        dtab[b * SR + r] = (short)max(d, -1100);   // 2^-1100 underflows to 0 in FP64
      }
    }
  }
  short* const ltab = dtab + (size_t)nbk * SR;    // LN: [np / XB][LR] Lambda exponents (<= 0)
  if constexpr (LN) {
    const int lrow0 = (PASS == 1) ? col0 : row0;
    const int* kl = p.kexpL + (size_t)lrow0 * nbk;
    for (int idx = tid; idx < LR * nbk; idx += C::THREADS) {
      const int r = idx / nbk, b = idx - r * nbk;
      ltab[b * LR + r] = (short)max(kl[(size_t)r * nbk + b], -1100);
    }
  }
  vm_wait<0>();
  __syncthreads();
#pragma unroll
  for (int kk = 1; kk < NBUF - 1; ++kk)
    if (kk < nks) stage_load(kk, bufp(kk));

  // pass-2 epilogue inputs, prefetched so that their latency hides behind the K loop (FP32: issued
  // one step into the first stage, so that one wave's load issue overlaps the other wave's MFMAs)
  double la_v[CB][RB][4], fo_v[CB][RB][4];
  double ao_v[ADJ ? CB : 1][ADJ ? RB : 1][4], lb_v[ADJ ? CB : 1][ADJ ? RB : 1][4];
  double ln_v[ADJ ? CB : 1][ADJ ? RB : 1][4];
  constexpr bool LATE_PF = PASS == 2 && !ADJ && std::is_same<T, float>::value;
  auto epi_prefetch = [&]() {
    const double* lnm = p.lnmarg + (size_t)bz * p.sMarg;
    const double* pot = p.pot + (size_t)bz * plane;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int j = col0 + wn * C::WTN + cb * 16 + r16;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = row0 + wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const bool ok = i < n && j < n;
          const size_t o = (size_t)i * np + j;
          // (non-temporal: each is read once per launch, by this tile only)
          la_v[cb][rb][e] = ok ? __builtin_nontemporal_load(&lnm[o]) : 0.0;
          fo_v[cb][rb][e] = (ok && (ADJ || p.err_on)) ? __builtin_nontemporal_load(&pot[o]) : 0.0;
          if constexpr (ADJ) {
            ao_v[cb][rb][e] = (ok && p.adj_acc) ? p.adj_out[(size_t)bz * plane + o] : 0.0;
            lb_v[cb][rb][e] = (ok && p.adj_lb) ? p.adj_lb[(size_t)bz * plane + o] : 0.0;
            ln_v[cb][rb][e] = (ok && p.adj_next_L) ? p.adj_next_L[(size_t)bz * plane + o] : 0.0;
          }
        }
    }
  };
  if constexpr (PASS == 2 && !LATE_PF) epi_prefetch();

  // marginal-error partials of the preceding update, summed in index order by workgroup 0;
  // the first PEND_REG per thread are read now, the sum is formed in the epilogue
  constexpr int PEND_REG = 2;
  const bool pend_wg = PASS == 1 && p.pend_parts && blockIdx.x == 0 && blockIdx.y == 0;
  double pend_v[PEND_REG];
#pragma unroll
  for (int q = 0; q < PEND_REG; ++q) {
    const int t = tid + q * C::THREADS;
    pend_v[q] = (pend_wg && t < p.pend_tiles) ? p.pend_parts[(size_t)bz * p.pend_tiles + t] : 0.0;
  }

  // Two sets of block accumulators, alternating by exponent block, so that a finished block is
  // flushed (FP64 rescale and add) one step later, while the next block's MFMAs run into the
  // other set; the block's exponent differences are read from LDS when the block starts.
  constexpr int ND = (PASS == 1) ? RB * 4 : CB;   // distinct scaled rows per lane
  acc_t acc[2][RB][CB];
  f64x4 accd[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      acc[0][i][j] = acc_t{};
      acc[1][i][j] = acc_t{};
      accd[i][j] = f64x4{};
    }
  int dcur[ND], dprev[ND];
#pragma unroll
  for (int q = 0; q < ND; ++q) dcur[q] = dprev[q] = 0;
  // LN: Lambda's exponents of this lane's output columns (pass 1) or rows (pass 2)
  constexpr int NL = LN ? ((PASS == 1) ? CB : RB * 4) : 1;
  int lcur[NL], lprev[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) lcur[q] = lprev[q] = 0;
  // LN: the largest block scale 2^(K + KL) each output was formed from (the range check's
  // reference; without Lambda's exponents it is 2^0, the reference exponent's own block)
  int emx[LN ? RB : 1][LN ? CB : 1][4];
#pragma unroll
  for (int i = 0; i < (LN ? RB : 1); ++i)
#pragma unroll
    for (int j = 0; j < (LN ? CB : 1); ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) emx[i][j][e] = KSENT;
  auto lrow = [&](int q) -> int {
    return (PASS == 1) ? wn * C::WTN + q * 16 + r16 : wm * C::WTM + (q / 4) * 16 + Mma<T>::row(g, q % 4);
  };
  // exponent that scales accumulator element (rb, cb, e) of the block held in dprev / lprev
  auto fscale = [&](int rb, int cb, int e) -> int {
    const int dd = dprev[PASS == 1 ? rb * 4 + e : cb];
    if constexpr (LN) return dd + lprev[PASS == 1 ? cb : rb * 4 + e];
    return dd;
  };
  // scaled row of exponent-difference entry q of this lane
  auto srow = [&](int q) -> int {
    return (PASS == 1) ? wm * C::WTM + (q / 4) * 16 + Mma<T>::row(g, q % 4) : wn * C::WTN + q * 16 + r16;
  };

  // Main loop over K stages, NBUF LDS buffers (stage kt + NBUF - 1 is requested when stage kt
  // starts).  Within a stage the fragments of step h + FRAG_AHEAD are read while the MFMAs of
  // step h run; at the end of a stage the workgroup waits for the next stage, synchronises and
  // requests the next stage's first fragments.
  static_assert((NBUF * HPS) % (2 * HB) == 0, "block parity must repeat with the unrolled stages");
  const int arow = (wm * C::WTM + r16) * FROWB, brow = ((TZ ? 0 : BM) + wn * C::WTN + r16) * FROWB;
  const int sw = (g ^ r16) << 4;                  // slot of chunk 4h+g in this lane's rows, h = 0
  // TZ: table offset of this lane's Lambda fragments (pass 1: B fragment cb, pass 2: A fragment
  // rb) at the loop's first step; each step advances K by 4 EPC values, i.e. TZSTEP bytes (BF16x3:
  // each pair of steps, hi halves from the hi window and then lo halves from the lo window)
  constexpr int NTZ = PASS == 1 ? CB : RB;
  constexpr int TZSTEP = 64 * EPC;
  int tzo[NTZ];
#pragma unroll
  for (int q = 0; q < NTZ; ++q) {
    const int lr = (PASS == 1 ? wn * C::WTN : wm * C::WTM) + q * 16 + r16;
    tzo[q] = 16 * (g * EPC + LR - 1 - lr);
  }
  // fragment reads: step s (from the loop's first K) of stage buffer buf at slot offset so
  auto tz_frag = [&](int off, int s) -> u32x4 {
    if constexpr (PAIRED) return *(const u32x4*)(tzt + ((s & 1) ? tzlo : 0) + off + (s >> 1) * TZSTEP);
    return *(const u32x4*)(tzt + off + s * TZSTEP);
  };
  auto frag_a = [&](const unsigned char* buf, int rb, int so, int s) -> u32x4 {
    if constexpr (TZ && PASS == 2) return tz_frag(tzo[rb], s);
    return *(const u32x4*)(&buf[arow + rb * 16 * FROWB + so]);
  };
  auto frag_b = [&](const unsigned char* buf, int cb, int so, int s) -> u32x4 {
    if constexpr (TZ && PASS == 1) return tz_frag(tzo[cb], s);
    return *(const u32x4*)(&buf[brow + cb * 16 * FROWB + so]);
  };
  // fragments of PD consecutive steps are live: slot h % PD holds step h of the stage (the
  // fragments of step h + FA are requested at step h; a BF16x3 pair step also reads step h - 1)
  constexpr int FA = FRAG_AHEAD;
  constexpr int PD = FA + 1 + (PAIRED ? 1 : 0);
  static_assert(HPS >= PD, "a stage holds at least the fragments in flight");
  u32x4 fa[PD][RB], fb[PD][CB];
#pragma unroll
  for (int hs = 0; hs < FA; ++hs) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) fa[hs][rb] = frag_a(lds0, rb, sw ^ (hs << 6), hs);
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) fb[hs][cb] = frag_b(lds0, cb, sw ^ (hs << 6), hs);
  }
  for (int kt0 = 0; kt0 < nks; kt0 += NBUF)
#pragma unroll
  for (int jb = 0; jb < NBUF; ++jb) {                // stage kt uses buffer jb = kt mod NBUF
    const int kt = kt0 + jb;
    if (kt >= nks) break;
    const unsigned char* cur = bufp(jb);
    const bool more = kt + 1 < nks;
    const bool ahead = kt + NBUF - 1 < nks;        // a stage is requested NBUF - 1 ahead
    if (ahead) stage_load(kt + NBUF - 1, bufp((jb + NBUF - 1) % NBUF));
#pragma unroll
    for (int h = 0; h < HPS; ++h) {
      const int hl = jb * HPS + h;                 // step within the unrolled stages
      const int par = (hl / HB) & 1;               // accumulator set of this step's block
      const bool first = hl % HB == 0, lastb = (hl + 1) % HB == 0;
      const bool last = h + 1 == HPS;
      if (first) {
        const int blk = ((kt + k_lo) * HPS + h) / HB;
#pragma unroll
        for (int q = 0; q < ND; ++q) dcur[q] = dtab[blk * SR + srow(q)];
        if constexpr (LN) {
#pragma unroll
          for (int q = 0; q < NL; ++q) lcur[q] = ltab[blk * LR + lrow(q)];
        }
      }
      if (h + FA < HPS) {
        const int ha = h + FA;                     // step whose fragments are requested now
        const int so = sw ^ (ha << 6);             // chunk 4 ha + g
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) fa[ha % PD][rb] = frag_a(cur, rb, so, kt * HPS + ha);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) fb[ha % PD][cb] = frag_b(cur, cb, so, kt * HPS + ha);
      }
      // FP32: keep these reads ahead of this step's MFMAs (the scheduler would otherwise sink
      // them next to their use and expose the LDS latency; measured 2-3% per launch)
      if constexpr (std::is_same<T, float>::value) __builtin_amdgcn_sched_barrier(0);
      if constexpr (PAIRED) {
        // hi.hi on the hi step; hi.lo and lo.hi on the lo step (consecutive MFMAs go to
        // different accumulators)
        const int hc = h % PD, hp = (h + PD - 1) % PD;
        if (h % 2 == 0) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) Mma<T>::run(fa[hc][rb], fb[hc][cb], acc[par][rb][cb]);
        } else {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) Mma<T>::run(fa[hp][rb], fb[hc][cb], acc[par][rb][cb]);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) Mma<T>::run(fa[hc][rb], fb[hp][cb], acc[par][rb][cb]);
        }
      } else {
        // sub-products outermost: consecutive MFMAs go to different accumulators
#pragma unroll
        for (int q = 0; q < Mma<T>::NSUB; ++q)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) Mma<T>::sub(fa[h % PD][rb], fb[h % PD][cb], acc[par][rb][cb], q);
      }
      if constexpr (LATE_PF) {
        if (jb == 0 && h == 1)
          if (kt0 == 0) epi_prefetch();
      }
      if (first && !(kt == 0 && h == 0)) {
        // flush the previous block (other set) with its exact power-of-two scales
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              accd[rb][cb][e] += ldexp((double)acc[par ^ 1][rb][cb][e], fscale(rb, cb, e));
              if constexpr (LN) emx[rb][cb][e] = max(emx[rb][cb][e], fscale(rb, cb, e));
            }
            acc[par ^ 1][rb][cb] = acc_t{};
          }
      }
      if (lastb) {
#pragma unroll
        for (int q = 0; q < ND; ++q) dprev[q] = dcur[q];
#pragma unroll
        for (int q = 0; q < NL; ++q) lprev[q] = lcur[q];
      }
      if (last) {
        // stage kt+1 landed; the stages requested after it may stay in flight
        const int inflight = min(NBUF - 1, nks - 1 - kt);
        if (NBUF > 3 && inflight >= 3)
          vm_wait<(NBUF > 3 ? 2 * UPW : 0)>();
        else if (NBUF > 2 && inflight >= 2)
          vm_wait<(NBUF > 2 ? UPW : 0)>();
        else
          vm_wait<0>();
        // workgroup barrier without a memory fence (a fence would wait for the stage still in
        // flight); the compiler-only fences keep LDS accesses on their side of it
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_barrier();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (more) {
          const unsigned char* nxt = bufp((jb + 1) % NBUF);
#pragma unroll
          for (int hs = 0; hs < FA; ++hs) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) fa[hs][rb] = frag_a(nxt, rb, sw ^ (hs << 6), (kt + 1) * HPS + hs);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) fb[hs][cb] = frag_b(nxt, cb, sw ^ (hs << 6), (kt + 1) * HPS + hs);
          }
        }
      }
    }
  }
  {
    // flush the last block: it used set ((K steps - 1) / HB) & 1
    const int lastpar = (((nks * HPS) - 1) / HB) & 1;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double v = lastpar ? (double)acc[1][rb][cb][e] : (double)acc[0][rb][cb][e];
          accd[rb][cb][e] += ldexp((double)v, fscale(rb, cb, e));
          if constexpr (LN) emx[rb][cb][e] = max(emx[rb][cb][e], fscale(rb, cb, e));
        }
  }
  // range margins of the outputs (see range_margin): the largest block scale is 2^0 without
  // Lambda's exponents (the reference block of the row), 2^emx with them
  auto margin_of = [&](int rb, int cb, int e, double v) -> int {
    if constexpr (LN)
      return range_margin(v, emx[rb][cb][e]);
    else
      return range_margin(v, 0);
  };
  auto range_report = [&](int mmin) {
    if (!p.range_slots) return;
    mmin = wave_min_int(mmin);
    if (lane == 0 && mmin < INT_MAX) {
      // (atomics without a result on addresses no other wave uses: nothing waits for them)
      int* sl = p.range_slots + 2 * ((size_t)bz * p.range_spt + (size_t)(blockIdx.x + gridDim.x * blockIdx.y) * C::NW + wave);
      atomicMin(sl, mmin);
      if (mmin < p.range_thr) atomicMin(sl + 1, p.iter);
    }
  };

  // ---------------------------------------------------------------- epilogues
  // accd[rb][cb][e] belongs to output row row0 + wm*WTM + rb*16 + Mma<T>::row(g, e) and column
  // col0 + wn*WTN + cb*16 + r16; its true value is accd * 2^(reference exponent).  The element
  // work is written without branches (selects), so the compiler interleaves the elements.
  if constexpr (PASS == 1) {
    // W[L][k] = accd 2^{R_L}.  Column block exponent K'[k] = max over the tile's XB1 rows of the
    // binary exponent of W; Bt[k][L] = W 2^{-K'} in (0, 1).
    int ecol[CB];
    int mmin = INT_MAX;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) ecol[cb] = KSENT;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int lr = wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const int i = row0 + lr, j = col0 + wn * C::WTN + cb * 16 + r16;
          const double v = accd[rb][cb][e];
          int ex;
          (void)frexp(v, &ex);
          // (signed sums of a reverse half-step: the exponent of |W|)
          ecol[cb] = max(ecol[cb], (i < n && j < n && (ADJ ? v != 0.0 : v > 0.0)) ? rref[lr] + ex : KSENT);
          // a row with mass has a positive product with Lambda at every column
          if (!ADJ && i < n && j < n && rref[lr] != KSENT) mmin = min(mmin, margin_of(rb, cb, e, v));
        }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      ecol[cb] = max(ecol[cb], __shfl_xor(ecol[cb], 16, 64));
      ecol[cb] = max(ecol[cb], __shfl_xor(ecol[cb], 32, 64));
      if (g == 0) ered[wn * C::WTN + cb * 16 + r16][wm] = ecol[cb];
    }
    // pending marginal-error sum: entries beyond the prefetched ones, then per-wave sums
    double pend = 0.0;
    if (pend_wg) {
#pragma unroll
      for (int q = 0; q < PEND_REG; ++q) pend += pend_v[q];
      for (int t = tid + PEND_REG * C::THREADS; t < p.pend_tiles; t += C::THREADS)
        pend += p.pend_parts[(size_t)bz * p.pend_tiles + t];
      pend = wave_sum_dpp(pend);
      if (lane == 0) red[wave] = pend;
    }
    lds_barrier();
    if (pend_wg && tid == 0) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < C::NW; ++w) v += red[w];
      p.pend_out[bz] = v;
    }
    T* outT = (T*)p.outT + (size_t)bz * plane;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int lc = wn * C::WTN + cb * 16 + r16;
      const int j = col0 + lc;
      const int xblk = wm / WPB1;                   // this wave's exponent block of rows
      int K = ered[lc][xblk * WPB1];
#pragma unroll
      for (int w = 1; w < WPB1; ++w) K = max(K, ered[lc][xblk * WPB1 + w]);
      if (wm % WPB1 == 0 && g == 0 && j < n) p.kexpT[((size_t)bz * np + j) * p.nbT + tr * C::XS + xblk] = K;
      if (j >= n) continue;  // padded rows of Bt stay zero
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if constexpr (sizeof(T) == 8) {
          // FP64 rows g + 4e are not contiguous: element stores
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int lr = wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
            const int i = row0 + lr;
            const double v = (K == KSENT) ? 0.0 : ldexp(accd[rb][cb][e], rref[lr] - K);
            // (a reverse half-step also writes the zeros of the padded rows i >= n: its Bt buffer
            // is shared with other kernels)
            if (ADJ || i < n) {
              if constexpr (NT_OPS)
                __builtin_nontemporal_store(v, (double*)&outT[(size_t)j * np + i]);
              else
                outT[(size_t)j * np + i] = v;
            }
          }
        } else if constexpr (PAIRED) {
          // rows 4g .. 4g+3: one 8-byte store of their hi halves and one of their lo halves
          typedef __bf16 hv4 __attribute__((ext_vector_type(4)));
          const int lr0 = wm * C::WTM + rb * 16 + 4 * g;
          const int k0 = row0 + lr0;
          hv4 wh, wl;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int lr = lr0 + e;
            const double v = (K == KSENT || row0 + lr >= n) ? 0.0 : ldexp(accd[rb][cb][e], rref[lr] - K);
            const T x = cvt_op<T>(v);
            wh[e] = x.hi;
            wl[e] = x.lo;
          }
          __bf16* r = (__bf16*)(outT + (size_t)j * np) + 2 * (k0 & ~31) + (k0 & 31);
          *(hv4*)r = wh;
          *(hv4*)(r + 32) = wl;
        } else {
          // rows 4g .. 4g+3 are contiguous in Bt row j: one 16-byte (FP32) or 8-byte store
          typedef T tv4 __attribute__((ext_vector_type(4)));
          const int lr0 = wm * C::WTM + rb * 16 + 4 * g;
          tv4 w;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int lr = lr0 + e;
            const double v = (K == KSENT || row0 + lr >= n) ? 0.0 : ldexp(accd[rb][cb][e], rref[lr] - K);
            w[e] = (T)v;
          }
          if constexpr (NT_OPS)
            __builtin_nontemporal_store(w, (tv4*)(outT + (size_t)j * np + row0 + lr0));
          else
            *(tv4*)(outT + (size_t)j * np + row0 + lr0) = w;
        }
      }
    }
    // (the range atomics go last: the workgroup barriers above wait for every outstanding store)
    range_report(mmin);
  } else if constexpr (ADJ) {
    // reverse half-step: K(w) = accd 2^{R'_k} (signed); out = mask ? (acc ? out : 0) +
    // w e^{P/eps} K(w) : 0, formed as |accd| e^{P/eps} 2^{R'_k} in one piece so that neither
    // e^{P/eps} nor K(w) alone has to be representable
    double* out = p.adj_out + (size_t)bz * plane;
    double* lb = p.adj_lb ? p.adj_lb + (size_t)bz * plane : nullptr;
    const double csc = 1.0 / sqrt((double)n), inv_eps = p.inv_eps;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int lc = wn * C::WTN + cb * 16 + r16;
      const int j = col0 + lc;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = row0 + wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const bool ok = i < n && j < n;
          const double v = accd[rb][cb][e];
          double w = p.adj_scale;
          if (p.adj_coords & 1) w *= (double)(i - n / 2) * csc;
          if (p.adj_coords & 2) w *= (double)(j - n / 2) * csc;
          double val = 0.0;
          if (v != 0.0 && w != 0.0) {
            const double x = fo_v[cb][rb][e] * inv_eps;
            const double mag =
                (sizeof(T) == 8) ? mul_exp_fp64(fabs(v), x, rref[lc]) : mul_exp_op32(fabs(v), x, rref[lc]);
            val = ((v < 0.0) != (w < 0.0) ? -mag : mag) * fabs(w);
          }
          val += ao_v[cb][rb][e];
          const bool keep = la_v[cb][rb][e] > -INFINITY;
          if (ok) {
            if (!p.adj_next_L) out[(size_t)i * np + j] = keep ? val : 0.0;
            if (lb && keep) lb[(size_t)i * np + j] = fma(p.adj_lb_scale, val, lb_v[cb][rb][e]);
          }
          // log-magnitude of the next operand's element (k_adj_prep's h), -inf where it is zero
          const double vo = (ok && keep) ? val : 0.0;
          const double lg = (sizeof(T) == 8) ? log_fp64(fabs(vo)) : log_op32(fabs(vo));
          ln_v[cb][rb][e] = (vo != 0.0) ? lg - ln_v[cb][rb][e] : -INFINITY;
          lb_v[cb][rb][e] = vo;   // (its sign)
        }
    }
    if (p.adj_next_L) {
      // next pass-1 operand: the tile's columns are XS exponent blocks of its rows
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int k = KSENT;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) k = max(k, block_exponent(ln_v[cb][rb][e]));
          k = row16_max(k);
          if (r16 == 0) kred[wm * C::WTM + rb * 16 + Mma<T>::row(g, e)][wn] = k;
        }
      lds_barrier();
      T* nA = (T*)p.nextA + (size_t)bz * plane;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int lr = wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const int i = row0 + lr;
          const int xblk = wn / WPB2;               // this wave's exponent block of columns
          int K = kred[lr][xblk * WPB2];
#pragma unroll
          for (int w = 1; w < WPB2; ++w) K = max(K, kred[lr][xblk * WPB2 + w]);
          if (wn % WPB2 == 0 && r16 == 0 && i < n) p.kexpN[((size_t)bz * np + i) * p.nbA + tc * C::XS + xblk] = K;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int j = col0 + wn * C::WTN + cb * 16 + r16;
            const T x = block_operand<T>(ln_v[cb][rb][e], K);
            if (i < n && j < n) store_op<T>(nA + (size_t)i * np, j, lb_v[cb][rb][e] < 0.0 ? (T)(-x) : x);
          }
        }
    }
  } else {
    // S = accd 2^{R'_k};  f_new = eps (ln m - ln S) in FP64, the marginal-error partial of the
    // entering plan, and (optionally) the next pass-1 operand of f_new.
    const double eps = p.eps, inv_eps = p.inv_eps;
    double* pot = p.pot + (size_t)bz * plane;
    double* lns = p.lnS_out ? p.lnS_out + (size_t)bz * plane : nullptr;
    double err = 0.0;
    bool bad = false;
    int mmin = INT_MAX;
    double fnew_v[CB][RB][4];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int lc = wn * C::WTN + cb * 16 + r16;
      const int j = col0 + lc;
      const double shift = (double)rref[lc] * LN2;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = row0 + wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const bool ok = i < n && j < n;
          const double v = accd[rb][cb][e];
          // ln S: FP64 logarithm for FP64 operands; for the FP32-accumulated types a logarithm
          // as accurate as the sum itself
          const double lnS = shift + ((sizeof(T) == 8) ? log_fp64(v) : log_op32(v));
          const double la = la_v[cb][rb][e];
          const double fold = fo_v[cb][rb][e];
          const bool zm = la == -INFINITY;
          const double fnew = (ok && !zm) ? eps * (la - lnS) : -INFINITY;
          if (p.err_on) {
            // marginal-error term of the entering plan at this pixel.  Its mass there is
            // u_old S = exp(x), x = f_old/eps + ln S; the term is that mass on a zero-mass pixel,
            // elsewhere a |u_old / u_new - 1| = a |exp(d) - 1| with d = (f_old - f_new)/eps =
            // x - ln a, taken as exp(x) - a once d is large (e^d alone can overflow FP32 for
            // tiny a).  Every candidate is formed and one selected: no branches.
            const double x = fma(fold, inv_eps, lnS);
            const float tz = exp_err((float)x);
            const float df = (float)(x - la);
            const float av = exp_err((float)la);
            const float ta = (df < 10.0f) ? av * fabsf(expm1_err(df)) : tz - av;
            err += ok ? (double)(zm ? tz : ta) : 0.0;
          }
          bad = bad || (ok && !zm && !(fabs(fnew) < INFINITY));
          if (ok && !zm && rref[lc] != KSENT) mmin = min(mmin, margin_of(rb, cb, e, v));
          const size_t o = (size_t)i * np + j;
          if (ok) {
            __builtin_nontemporal_store(fnew, &pot[o]);   // (read again only a full iteration later)
            if (lns) lns[o] = lnS;
          }
          fnew_v[cb][rb][e] = fnew;
        }
    }
    if (bad) atomicOr(p.flag, 1);
    if (p.err_on) {
      err = wave_sum_dpp(err);
      if (lane == 0) red[wave] = err;
    }

    if (p.next_inv_eps > 0.0) {
      // next pass-1 operand: per output row, the exponent of the max over each XB2 of the tile's columns
      const double ninv = p.next_inv_eps;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int k = KSENT;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) k = max(k, block_exponent(fnew_v[cb][rb][e] * ninv));
          k = row16_max(k);   // over the 16 columns of this lane's block row
          if (r16 == 0) kred[wm * C::WTM + rb * 16 + Mma<T>::row(g, e)][wn] = k;
        }
    }
    lds_barrier();
    if (p.err_on && tid == 0) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < C::NW; ++w) v += red[w];
      // (indexed by tile, so that the fixed-order sum does not depend on the tile mapping)
      p.partials[(size_t)bz * gridDim.x * gridDim.y + tc + gridDim.x * tr] = v;
    }
    if (p.next_inv_eps > 0.0) {
      const double ninv = p.next_inv_eps;
      T* nA = (T*)p.nextA + (size_t)bz * plane;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int lr = wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const int i = row0 + lr;
          const int xblk = wn / WPB2;               // this wave's exponent block of columns
          int K = kred[lr][xblk * WPB2];
#pragma unroll
          for (int w = 1; w < WPB2; ++w) K = max(K, kred[lr][xblk * WPB2 + w]);
          if (wn % WPB2 == 0 && r16 == 0 && i < n) p.kexpN[((size_t)bz * np + i) * p.nbA + tc * C::XS + xblk] = K;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int j = col0 + wn * C::WTN + cb * 16 + r16;
            const T x = block_operand<T>(fnew_v[cb][rb][e] * ninv, K);
            if (i < n && j < n) {
              if constexpr (NT_OPS)
                __builtin_nontemporal_store(x, nA + (size_t)i * np + j);
              else
                store_op<T>(nA + (size_t)i * np, j, x);
            }
          }
        }
    }
    range_report(mmin);   // (last: the workgroup barriers above wait for every outstanding store)
  }
}

}  // namespace fot
