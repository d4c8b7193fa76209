// Whole half-steps of the FOT iteration in one launch, for small grids (gfx950).
//
// One half-step of Algorithm 1 (arXiv 2512.19072, Sec. 3, Eq. 7 or Eq. 8) computes
// S = Lambda . exp(P/eps) . Lambda and the new potential eps (ln m - ln S).  The output columns
// k of S depend only on the same columns of the first product W = At . Lambda^T (all its rows),
// so one workgroup can own a panel of 32 output columns and run both per-axis products for it:
//
//   pass 1  W[:, panel] = At . Lambda[panel, :]^T        (all n_p rows, 32 columns; kept in LDS,
//                                                          transposed and block-normalised)
//   pass 2  S[:, panel] = Lambda . W[:, panel]            (all n_p rows, 32 columns)
//
// followed by the epilogue of the fused pass-2 kernel (FP64 potential update, marginal-error
// partial, next pass-1 operand with its block exponents, range margins).  A half-step is then
// one launch of n_p / 32 workgroups instead of two dependent launches, which is what bounds the
// iteration time on grids of a few hundred pixels.  The operand formats are those of the 32 x 32
// fused kernels (exponent blocks of 32), so either kernel can follow the other.  Raw (not block-
// normalised) Lambda only; FP32, BF16 and FP16 operands.
#pragma once

#include "fot_fused.hpp"

namespace fot {

constexpr int PANEL = 32;          // output columns per workgroup = exponent block width
constexpr int PANEL_THREADS = 256; // four waves, one per SIMD
constexpr int PANEL_MAX_NP = 256;  // largest padded side (LDS and latency budget)

struct PanelArgs {
  const void* A;            // [batch][np][np] block-normalised pass-1 operand (blocks of 32 columns)
  const int* kexpA;         // [batch][np][np / 32] its exponents
  const void* lam;          // [np][np] Lambda in the operand type (raw form)
  int n, np, nb;            // valid side, padded side, np / 32
  int band;                 // Lambda[i][k] is zero in the operand type for |i - k| > band
  const double* lnmarg;     // ln a or ln b, [np][np] with batch stride sMarg
  long long sMarg;
  double* pot;              // potential updated in place
  double* lnS_out;          // optional copy of ln S
  double eps, inv_eps;
  double next_inv_eps;      // > 0: also write the next pass-1 operand with this 1/eps
  void* nextA;              // [batch][np][np]
  int* kexpN;               // [batch][np][np / 32]
  double* partials;         // [batch][np / 32] marginal-error partials of this half-step
  int* flag;
  int err_on;
  const double* pend_parts; // partials of the preceding half-step (nullptr: none), summed by panel 0
  int pend_tiles;
  double* pend_out;
  int* range_iter;          // as FusedArgs
  int iter;
  int* range_min;
  int range_thr;
};

// LDS of one panel workgroup: row reference exponents and exponent differences of the pass-1
// operand, the block-normalised transposed intermediate Bt[32][np + pad] with its exponents.
template <typename T>
struct PanelLds {
  static constexpr int PAD = 16 / (int)sizeof(T);   // one 16-byte slot per row: conflict-free reads
  static size_t bytes(int np) {
    const int nb = np / PANEL;
    return (size_t)np * sizeof(int) + (size_t)nb * np * sizeof(short) + (size_t)PANEL * nb * sizeof(int) +
           PANEL * sizeof(int) + (size_t)PANEL * (np + PAD) * sizeof(T);
  }
};

template <typename T>
__global__ __launch_bounds__(PANEL_THREADS) void k_panel(const PanelArgs p) {
  typedef typename Mma<T>::acc_t acc_t;
  static_assert(!Mma<T>::PAIRED && sizeof(T) <= 4, "FP32, BF16 and FP16 operands");
  constexpr int EPH = 64 / (int)sizeof(T);     // K values per fragment step (4 lane groups)
  constexpr int HB = PANEL / EPH;              // fragment steps per exponent block
  constexpr int PAD = PanelLds<T>::PAD;
  extern __shared__ __attribute__((aligned(16))) unsigned char plds[];
  const int np = p.np, n = p.n, nb = p.nb;
  int* rref = (int*)plds;                                   // [np]
  short* dtab = (short*)(rref + np);                        // [nb][np]
  int* ktab = (int*)(dtab + (size_t)nb * np);               // [PANEL][nb]: K' then K' - kref2
  int* kref2 = ktab + PANEL * nb;                           // [PANEL]
  T* bt = (T*)(kref2 + PANEL);                              // [PANEL][np + PAD]
  __shared__ double red[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int bz = blockIdx.z, panel = blockIdx.x, col0 = panel * PANEL;
  const size_t plane = (size_t)np * np;
  const int ldb = np + PAD;

  // the preceding half-step's marginal-error partials (another buffer than this launch writes)
  if (p.pend_parts && panel == 0) {
    double v = 0.0;
    for (int t = tid; t < p.pend_tiles; t += PANEL_THREADS) v += p.pend_parts[(size_t)bz * p.pend_tiles + t];
    v = wave_sum_dpp(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (tid == 0) p.pend_out[bz] = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
  }

  // pass-1 operand exponents: reference (largest block exponent) of every row, and each block's
  // difference to it (2^-1100 underflows to 0 in FP64)
  {
    const int* kx = p.kexpA + (size_t)bz * np * nb;
    for (int r = tid; r < np; r += PANEL_THREADS) {
      int m = KSENT;
      for (int b = 0; b < nb; ++b) m = max(m, kx[(size_t)r * nb + b]);
      rref[r] = m;
      for (int b = 0; b < nb; ++b) dtab[(size_t)b * np + r] = (short)max(kx[(size_t)r * nb + b] - m, -1100);
    }
  }
  __syncthreads();

  const unsigned char* Ab = (const unsigned char*)p.A + (size_t)bz * plane * sizeof(T);
  const unsigned char* Lb = (const unsigned char*)p.lam;
  const size_t pitch = (size_t)np * sizeof(T);
  // lane's 16-byte chunk of a fragment step at K offset kk: row r, elements kk + g EPH/4 ...
  auto frag = [&](const unsigned char* base, int r, int kk) -> u32x4 {
    return *(const u32x4*)(base + (size_t)r * pitch + (size_t)(kk + g * (EPH / 4)) * sizeof(T));
  };
  // the K blocks of 32 whose Lambda entries can be nonzero for rows (or columns) [r0, r0 + 32)
  auto block_in_band = [&](int b, int r0) -> bool {
    return p.band >= n || (PANEL * b <= r0 + PANEL - 1 + p.band && PANEL * b + PANEL - 1 >= r0 - p.band);
  };
  constexpr int RANGE_NONE = INT_MAX;
  int mmin = RANGE_NONE;

  // ------------------------------------------------------------ pass 1: W[:, panel], to LDS
  for (int rg = wave; rg < np / PANEL; rg += 4) {
    const int row0 = rg * PANEL;
    acc_t acc[2][2];
    f64x4 accd[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) accd[i][j] = f64x4{};
    for (int b = 0; b < nb; ++b) {
      if (!block_in_band(b, col0)) continue;    // Lambda rows of the panel vanish on this block
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{};
#pragma unroll
      for (int h = 0; h < HB; ++h) {
        const int kk = b * PANEL + h * EPH;
        u32x4 fa[2], fb[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) fa[rb] = frag(Ab, row0 + rb * 16 + r16, kk);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) fb[cb] = frag(Lb, col0 + cb * 16 + r16, kk);
#pragma unroll
        for (int q = 0; q < Mma<T>::NSUB; ++q)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) Mma<T>::sub(fa[rb], fb[cb], acc[rb][cb], q);
      }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int d = dtab[(size_t)b * np + row0 + rb * 16 + Mma<T>::row(g, e)];
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) accd[rb][cb][e] += ldexp((double)acc[rb][cb][e], d);
        }
    }
    // W = accd 2^{rref}.  Exponent K'[k][rg] of each column over this block of rows; Bt[k][L] =
    // W 2^{-K'} in the operand type; range margins of rows with mass.
    int ecol[2] = {KSENT, KSENT};
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = row0 + rb * 16 + Mma<T>::row(g, e), j = col0 + cb * 16 + r16;
          const double v = accd[rb][cb][e];
          int ex;
          (void)frexp(v, &ex);
          const bool live = i < n && j < n && rref[i] != KSENT;
          ecol[cb] = max(ecol[cb], (live && v > 0.0) ? rref[i] + ex : KSENT);
          if (live) mmin = min(mmin, range_margin(v, 0));
        }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      ecol[cb] = max(ecol[cb], __shfl_xor(ecol[cb], 16, 64));
      ecol[cb] = max(ecol[cb], __shfl_xor(ecol[cb], 32, 64));
      if (g == 0) ktab[(cb * 16 + r16) * nb + rg] = ecol[cb];
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int K = ecol[cb];
      const int cl = cb * 16 + r16;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        // rows 4g .. 4g+3 are contiguous in Bt row cl
        typedef T tv4 __attribute__((ext_vector_type(4)));
        const int lr0 = row0 + rb * 16 + 4 * g;
        tv4 w;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = lr0 + e;
          const double v = (K == KSENT || i >= n || rref[i] == KSENT) ? 0.0 : ldexp(accd[rb][cb][e], rref[i] - K);
          w[e] = (T)v;   // rounded as the fused pass 1 rounds its transposed store
        }
        *(tv4*)(bt + (size_t)cl * ldb + lr0) = w;
      }
    }
  }
  __syncthreads();
  // reference exponent of each panel column, and each row block's difference to it
  if (tid < PANEL) {
    int m = KSENT;
    for (int b = 0; b < nb; ++b) m = max(m, ktab[tid * nb + b]);
    kref2[tid] = m;
    for (int b = 0; b < nb; ++b) ktab[tid * nb + b] = max(ktab[tid * nb + b] - m, -1100);
  }
  __syncthreads();

  // ------------------------------------------------------------ pass 2: S[:, panel] and epilogue
  const double eps = p.eps, inv_eps = p.inv_eps;
  double* pot = p.pot + (size_t)bz * plane;
  double* lns = p.lnS_out ? p.lnS_out + (size_t)bz * plane : nullptr;
  const double* lnm = p.lnmarg + (size_t)bz * p.sMarg;
  T* nA = (T*)p.nextA + (size_t)bz * plane;
  double err = 0.0;
  bool bad = false;
  for (int rg = wave; rg < np / PANEL; rg += 4) {
    const int j0 = rg * PANEL;
    acc_t acc[2][2];
    f64x4 accd[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) accd[i][j] = f64x4{};
    for (int b = 0; b < nb; ++b) {
      if (!block_in_band(b, j0)) continue;      // Lambda rows j0 .. j0+31 vanish on this block
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{};
#pragma unroll
      for (int h = 0; h < HB; ++h) {
        const int kk = b * PANEL + h * EPH;
        u32x4 fa[2], fb[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) fa[rb] = frag(Lb, j0 + rb * 16 + r16, kk);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          fb[cb] = *(const u32x4*)(bt + (size_t)(cb * 16 + r16) * ldb + kk + g * (EPH / 4));
#pragma unroll
        for (int q = 0; q < Mma<T>::NSUB; ++q)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) Mma<T>::sub(fa[rb], fb[cb], acc[rb][cb], q);
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int d = ktab[(cb * 16 + r16) * nb + b];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int e = 0; e < 4; ++e) accd[rb][cb][e] += ldexp((double)acc[rb][cb][e], d);
      }
    }
    // S = accd 2^{kref2}; f_new = eps (ln m - ln S) in FP64, the marginal-error term of the
    // entering plan, the next pass-1 operand of f_new (this panel is one exponent block of it)
    double fnew_v[2][2][4];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int cl = cb * 16 + r16, j = col0 + cl;
      const double shift = (double)kref2[cl] * LN2;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = j0 + rb * 16 + Mma<T>::row(g, e);
          const bool ok = i < n && j < n;
          const size_t o = (size_t)i * np + j;
          const double v = accd[rb][cb][e];
          const double lnS = shift + log_op32(v);
          const double la = ok ? lnm[o] : 0.0;
          const double fold = (ok && p.err_on) ? pot[o] : 0.0;
          const bool zm = la == -INFINITY;
          const double fnew = (ok && !zm) ? eps * (la - lnS) : -INFINITY;
          if (p.err_on) {
            // as in the fused pass 2: u_old S on a zero-mass pixel, a |exp(d) - 1| elsewhere
            const float tz = exp_err((float)fma(fold, inv_eps, lnS));
            const double d = (fold - fnew) * inv_eps;
            const float df = (float)d, laf = (float)la;
            const float av = exp_err(laf);
            const float ta = (df < 10.0f) ? av * fabsf(expm1_err(df)) : exp_err(laf + df) - av;
            err += ok ? (double)(zm ? tz : ta) : 0.0;
          }
          bad = bad || (ok && !zm && !(fabs(fnew) < INFINITY));
          if (ok && !zm && kref2[cl] != KSENT) mmin = min(mmin, range_margin(v, 0));
          if (ok) {
            pot[o] = fnew;
            if (lns) lns[o] = lnS;
          }
          fnew_v[rb][cb][e] = fnew;
        }
    }
    if (p.next_inv_eps > 0.0) {
      const double ninv = p.next_inv_eps;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = j0 + rb * 16 + Mma<T>::row(g, e);
          int K = max(block_exponent(fnew_v[rb][0][e] * ninv), block_exponent(fnew_v[rb][1][e] * ninv));
          K = row16_max(K);   // over the 16 columns of this lane's row in each half of the panel
          if (r16 == 0 && i < n) p.kexpN[((size_t)bz * np + i) * nb + panel] = K;
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) {
            const int j = col0 + cb * 16 + r16;
            if (i < n && j < n) store_op<T>(nA + (size_t)i * np, j, block_operand<T>(fnew_v[rb][cb][e] * ninv, K));
          }
        }
    }
  }
  if (bad) atomicOr(p.flag, 1);
  if (p.range_min) {
    const int m = wave_min_int(mmin);
    if (lane == 0 && m < RANGE_NONE) {
      atomicMin(p.range_min + bz, m);
      if (m < p.range_thr) atomicMin(p.range_iter + bz, p.iter);
    }
  }
  if (p.err_on) {
    err = wave_sum_dpp(err);
    __syncthreads();
    if (lane == 0) red[wave] = err;
    __syncthreads();
    if (tid == 0) p.partials[(size_t)bz * gridDim.x + panel] = red[0] + red[1] + red[2] + red[3];
  }
}

}  // namespace fot
