// Fused half-step of the FOT iteration for gfx950: two kernels per half-step.
//
// One half-step of Algorithm 1 (arXiv 2512.19072, Sec. 3, Eq. 7 or Eq. 8) computes, in the log
// domain, ln S = ln(Lambda . exp(P/eps) . Lambda) and the new potential eps (ln m - ln S).
// Every operand the per-axis GEMMs consume is stored normalised per 64-wide block of its K
// index by an integer power of two:
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
//   pass 2  S~ = Lambda . Bt^T, ln S = R'_k ln 2 + ln S~; epilogue updates the potential, the
//           marginal-error partial, and writes the next pass-1 operand At and its exponents.
#pragma once

#include "fot_kernels.hpp"

namespace fot {

constexpr int XBLK = 64;                  // K extent of one exponent block
constexpr int KSENT = -(1 << 20);          // exponent of an all-zero block
constexpr double LN2 = 0.69314718055994530942;
constexpr double INV_LN2 = 1.44269504088896340736;

struct FusedArgs {
  const void* A;            // [batch][np][np] pass-1: At;  pass-2: Lambda (shared, sA = 0)
  const void* B;            // [batch][np][np] pass-1: Lambda (shared); pass-2: Bt
  long long sA, sB;
  int n, np, nk, nb;        // nb = np / XBLK exponent blocks per row
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
};

// exp(x - K ln 2) rounded to the operand type, with the K of a block's maximum.  The prep
// kernel and the pass-2 epilogue both use these two functions, so the operand built after a
// replay from a checkpoint is bit-identical to the one built inside the iteration.
__device__ __forceinline__ int block_exponent(double xmax) {
  return (xmax > -INFINITY) ? (int)ceil(xmax * INV_LN2) : KSENT;
}
template <typename T>
__device__ __forceinline__ T block_operand(double x, int K) {
  return (K == KSENT) ? (T)0 : exp_op<T>(x - (double)K * LN2);
}

// Block-normalised pass-1 operand of a potential P (FP64 [batch][np][np]): one wave per row.
template <typename T>
__global__ __launch_bounds__(64) void k_prep_blocks(const double* P, int n, int np, double inv_eps, T* out,
                                                    int* kexp) {
  const int j = blockIdx.x, bz = blockIdx.y, lane = threadIdx.x;
  const int nb = np / XBLK;
  const size_t plane = (size_t)np * np;
  T* o = out + bz * plane + (size_t)j * np;
  int* ko = kexp + ((size_t)bz * np + j) * nb;
  for (int blk = 0; blk < nb; ++blk) {
    const int k = blk * XBLK + lane;
    const bool ok = j < n && k < n;
    const double x = ok ? P[bz * plane + (size_t)j * np + k] * inv_eps : -INFINITY;
    const int K = block_exponent(wave_max(x));
    o[k] = ok ? block_operand<T>(x, K) : (T)0;
    if (lane == 0) ko[blk] = K;
  }
}

template <typename T, int PASS, typename C>
__global__ __launch_bounds__(C::THREADS) void k_fused(const FusedArgs p) {
  static_assert(C::BM == XBLK && C::BN == XBLK, "exponent blocks are the 64-wide output tiles");
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int BM = C::BM, BN = C::BN, RB = C::RB, CB = C::CB;
  constexpr int HPS = CHUNKS / 4;                 // fragment steps per K stage
  constexpr int EPH = 64 / (int)sizeof(T);        // K elements per fragment step (4 lane groups)
  constexpr int HB = XBLK / EPH;                  // fragment steps per exponent block
  constexpr int MAXNB = 128;                      // np <= 8192
  __shared__ __attribute__((aligned(16))) unsigned char ldsA[2][BM * LDS_RS];
  __shared__ __attribute__((aligned(16))) unsigned char ldsB[2][BN * LDS_RS];
  __shared__ short dtab[MAXNB][XBLK];             // exponent - row reference, per block
  __shared__ int rref[XBLK];                      // reference exponent of each scaled row
  __shared__ double red[C::NW];
  __shared__ double xred[C::WGN][BM];             // pass 2: row maxima of the next operand
  __shared__ int ered[C::WGM][BN];                // pass 1: column exponent maxima

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / C::WGN, wn = wave % C::WGN;
  const int r16 = lane & 15, g = lane >> 4;
  const int bz = blockIdx.z;
  const int n = p.n, np = p.np, nb = p.nb;
  int tr, tc;
  tile_of(gridDim.x, gridDim.y, p.xcd_swizzle, &tr, &tc);
  const int row0 = tr * BM, col0 = tc * BN;
  const size_t plane = (size_t)np * np;

  // ---- exponent table of the block-normalised operand for this tile's 64 scaled rows
  // (pass 1: A rows = output rows; pass 2: B rows = output columns)
  {
    const int srow0 = (PASS == 1) ? row0 : col0;
    const int* kx = p.kexp + ((size_t)bz * np + srow0) * nb;
    for (int r = tid / 8; r < XBLK; r += C::THREADS / 8) {
      const int sub = tid % 8;
      int m = KSENT;
      for (int b = sub; b < nb; b += 8) m = max(m, kx[(size_t)r * nb + b]);
      m = max(m, __shfl_xor(m, 1, 64));
      m = max(m, __shfl_xor(m, 2, 64));
      m = max(m, __shfl_xor(m, 4, 64));
      if (sub == 0) rref[r] = m;
      for (int b = sub; b < nb; b += 8) {
        const int d = kx[(size_t)r * nb + b] - m;
        dtab[b][r] = (short)max(d, -1100);     // 2^-1100 underflows to 0 in FP64
      }
    }
  }

  const size_t pitch = (size_t)np * sizeof(T);
  const unsigned char* Ab = (const unsigned char*)p.A + ((size_t)bz * p.sA) * sizeof(T) + (size_t)row0 * pitch;
  const unsigned char* Bb = (const unsigned char*)p.B + ((size_t)bz * p.sB) * sizeof(T) + (size_t)col0 * pitch;
  constexpr int LA = BM * CHUNKS / C::THREADS, LB = BN * CHUNKS / C::THREADS;
  constexpr int RSTEP = C::THREADS / CHUNKS;
  const int rl = tid / CHUNKS, ql = tid % CHUNKS;
  const unsigned char* Ag = Ab + (size_t)rl * pitch + (size_t)ql * 16;
  const unsigned char* Bg = Bb + (size_t)rl * pitch + (size_t)ql * 16;
  const int sofs = rl * LDS_RS + ql * 16;
  u32x4 ga[LA], gb[LB];

  acc_t acc[RB][CB];
  f64x4 accd[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      acc[i][j] = acc_t{};
      accd[i][j] = f64x4{};
    }

  // pass-2 epilogue inputs, prefetched so that their latency hides behind the K loop
  double la_v[CB][RB][4], fo_v[CB][RB][4];
  if constexpr (PASS == 2) {
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
          la_v[cb][rb][e] = ok ? lnm[o] : 0.0;
          fo_v[cb][rb][e] = ok ? pot[o] : 0.0;
        }
    }
  }

  // marginal-error sum of the preceding update, finished in index order by one workgroup
  if constexpr (PASS == 1) {
    if (p.pend_parts && blockIdx.x == 0 && blockIdx.y == 0) {
      double v = 0.0;
      for (int t = tid; t < p.pend_tiles; t += C::THREADS) v += p.pend_parts[(size_t)bz * p.pend_tiles + t];
      v = block_sum(v, red);
      if (tid == 0) p.pend_out[bz] = v;
    }
  }

#pragma unroll
  for (int u = 0; u < LA; ++u) ga[u] = *(const u32x4*)(Ag + (size_t)u * RSTEP * pitch);
#pragma unroll
  for (int u = 0; u < LB; ++u) gb[u] = *(const u32x4*)(Bg + (size_t)u * RSTEP * pitch);
#pragma unroll
  for (int u = 0; u < LA; ++u) *(u32x4*)(&ldsA[0][sofs + u * RSTEP * LDS_RS]) = ga[u];
#pragma unroll
  for (int u = 0; u < LB; ++u) *(u32x4*)(&ldsB[0][sofs + u * RSTEP * LDS_RS]) = gb[u];
  __syncthreads();
  for (int kt = 0; kt < p.nk; ++kt) {
    const int s = kt & 1;
    const bool more = kt + 1 < p.nk;
    if (more) {
      const size_t ko = (size_t)(kt + 1) * ROWB;
#pragma unroll
      for (int u = 0; u < LA; ++u) ga[u] = *(const u32x4*)(Ag + (size_t)u * RSTEP * pitch + ko);
#pragma unroll
      for (int u = 0; u < LB; ++u) gb[u] = *(const u32x4*)(Bg + (size_t)u * RSTEP * pitch + ko);
    }
#pragma unroll
    for (int h = 0; h < HPS; ++h) {
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
      const int hh = kt * HPS + h;
      if ((hh + 1) % HB == 0) {
        // end of an exponent block: add its partial sums, scaled exactly by 2^(K - Kref)
        const int blk = hh / HB;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int sr = (PASS == 1) ? wm * C::WTM + rb * 16 + Mma<T>::row(g, e) : wn * C::WTN + cb * 16 + r16;
              accd[rb][cb][e] += ldexp((double)acc[rb][cb][e], (int)dtab[blk][sr]);
            }
            acc[rb][cb] = acc_t{};
          }
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
  // accd[rb][cb][e] belongs to output row row0 + wm*WTM + rb*16 + Mma<T>::row(g, e) and column
  // col0 + wn*WTN + cb*16 + r16; its true value is accd * 2^(reference exponent).
  if constexpr (PASS == 1) {
    // W[L][k] = accd 2^{R_L}.  Column block exponent K'[k] = max over this tile's rows of the
    // binary exponent of W; Bt[k][L] = W 2^{-K'} in (0, 1).
    int ecol[CB];
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
          if (i < n && j < n && v > 0.0) {
            int ex;
            (void)frexp(v, &ex);
            ecol[cb] = max(ecol[cb], rref[lr] + ex);
          }
        }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      ecol[cb] = max(ecol[cb], __shfl_xor(ecol[cb], 16, 64));
      ecol[cb] = max(ecol[cb], __shfl_xor(ecol[cb], 32, 64));
      if (g == 0) ered[wm][wn * C::WTN + cb * 16 + r16] = ecol[cb];
    }
    __syncthreads();
    T* outT = (T*)p.outT + (size_t)bz * plane;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int lc = wn * C::WTN + cb * 16 + r16;
      const int j = col0 + lc;
      int K = ered[0][lc];
#pragma unroll
      for (int w = 1; w < C::WGM; ++w) K = max(K, ered[w][lc]);
      if (wm == 0 && g == 0 && j < n) p.kexpT[((size_t)bz * np + j) * nb + tr] = K;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int lr = wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const int i = row0 + lr;
          if (i < n && j < n) {
            const double v = (K == KSENT) ? 0.0 : ldexp(accd[rb][cb][e], rref[lr] - K);
            outT[(size_t)j * np + i] = (T)v;
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
    int bad = 0;
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
          double fnew = -INFINITY;
          if (i < n && j < n) {
            const size_t o = (size_t)i * np + j;
            const double v = accd[rb][cb][e];
            // ln S: FP64 log for FP32/FP64 operands, logf for 16-bit operands
            const double lnS = shift + ((sizeof(T) == 2) ? (double)logf((float)v) : log(v));
            const double la = la_v[cb][rb][e];
            const double fold = fo_v[cb][rb][e];
            if (la == -INFINITY) {
              // entering plan's mass on a zero-mass pixel: u_old * S
              err += (double)expf((float)(fold * inv_eps + lnS));
            } else {
              fnew = eps * (la - lnS);
              // a |u_old / u_new - 1| = a |exp((f_old - f_new)/eps) - 1|
              err += (double)(expf((float)la) * fabsf(expm1f((float)((fold - fnew) * inv_eps))));
              bad |= !(fabs(fnew) < INFINITY);
            }
            pot[o] = fnew;
            if (lns) lns[o] = lnS;
          }
          fnew_v[cb][rb][e] = fnew;
        }
    }
    if (bad) atomicOr(p.flag, 1);
    const double part = block_sum(err, red);
    const int tiles = gridDim.x * gridDim.y;
    if (tid == 0) p.partials[(size_t)bz * tiles + blockIdx.x + gridDim.x * blockIdx.y] = part;

    if (p.next_inv_eps > 0.0) {
      // next pass-1 operand: per output row, exponent of the max over this tile's 64 columns
      const double ninv = p.next_inv_eps;
      double xm[RB][4];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          double m = -INFINITY;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) m = fmax(m, fnew_v[cb][rb][e] * ninv);
          m = fmax(m, __shfl_xor(m, 1, 64));
          m = fmax(m, __shfl_xor(m, 2, 64));
          m = fmax(m, __shfl_xor(m, 4, 64));
          m = fmax(m, __shfl_xor(m, 8, 64));
          xm[rb][e] = m;
          if (r16 == 0) xred[wn][wm * C::WTM + rb * 16 + Mma<T>::row(g, e)] = m;
        }
      __syncthreads();
      T* nA = (T*)p.nextA + (size_t)bz * plane;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int lr = wm * C::WTM + rb * 16 + Mma<T>::row(g, e);
          const int i = row0 + lr;
          double m = xred[0][lr];
#pragma unroll
          for (int w = 1; w < C::WGN; ++w) m = fmax(m, xred[w][lr]);
          const int K = block_exponent(m);
          if (wn == 0 && r16 == 0 && i < n) p.kexpN[((size_t)bz * np + i) * nb + tc] = K;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int j = col0 + wn * C::WTN + cb * 16 + r16;
            if (i < n && j < n) nA[(size_t)i * np + j] = block_operand<T>(fnew_v[cb][rb][e] * ninv, K);
          }
        }
      (void)xm;
    }
  }
}

}  // namespace fot
