// cFOT for gfx950: the Gibbs-kernel application of Algorithm 1 as linear convolutions
// (arXiv 2512.19072, Sec. 3, convolutional speedup, Eq. 11): Lambda is Toeplitz, so
// Lambda . V . Lambda = lambda * V * lambda with lambda_j = exp(-j^2 / (2 n^2 eps)),
// j = -(n-1) .. n-1, each 1-D convolution evaluated by FP64 FFTs of length N >= 2n - 1.
//
// One half-step is two row passes.  A pass takes each row of its input in the log domain,
// shifts it by the row maximum (exact: the shift factors out of the row's convolution),
// exponentiates, convolves with lambda by FFT and writes ln of the result transposed, so the
// second pass convolves the other axis by reading rows again:
//
//   pass 1  Yt[k][L] = m_L + ln sum_M exp(P[L][M]/eps - m_L) lambda(M - k)
//   pass 2  ln S[j][k] = m'_k + ln sum_L exp(Yt[k][L] - m'_k) lambda(L - j), stored as row k
//
// so a half-step maps a potential stored in one orientation to the next potential stored in the
// other: psi lives in natural layout [L][M], f transposed [k][j] (with ln a transposed to match),
// and the u-update (input psi) writes f^T while the V-update (input f^T) writes psi.
//
// Each workgroup transforms two rows at once as the real and imaginary parts of one complex
// sequence (lambda's transform is real and even, so the two results stay separate), entirely in
// LDS, by a mixed-radix Stockham FFT (natural order in and out): each stage reads R values per
// work item with stride N/R, applies the stage twiddles, runs a radix-R DFT in registers
// (R = 8, with one radix-4 or radix-2 stage last) and writes the R results with stride Ns, the
// product of the radices done so far.  N = 2^k is a compile-time parameter (256 .. 4096), so
// every index is a shift or a mask and the register arrays are fixed.
//
// Accuracy: an FFT's rounding is relative to the whole row, so a convolution value far below its
// row's largest carries an absolute error of about 1e-16 of that row's sum.  This is the source of
// the cFOT instability the paper reports at small eps (Sec. 4): ln of a tiny or (by rounding)
// non-positive value.  Non-positive values give -inf here, which the potential update reports as
// a non-finite potential.
#pragma once

#include "fot_fused.hpp"

namespace fot {

struct cplx {
  double re, im;
};

constexpr int CFOT_THREADS = 256;
constexpr int CFOT_MIN_N = 256;    // FFT lengths: powers of two in [256, 4096] (n <= 2048)
constexpr int CFOT_MAX_N = 4096;

// The Stockham stages of a length-N transform have sub-transform sizes NS = 1, 8, 64, ... (< N)
// and radix R = min(8, N / NS).  Stage NS > 1 multiplies its work item j by the powers of
// w = exp(-2 pi i (j mod NS) / (NS R)); the base twiddles of all stages sit in one table,
// stage NS at offset cfot_tw_offset(NS), indexed by j mod NS (contiguous across a wave).
constexpr int cfot_tw_offset(int NS) {
  int off = 0;
  for (int ns = 8; ns < NS; ns *= 8) off += ns;
  return off;
}
constexpr int cfot_tw_count(int N) { return cfot_tw_offset(N); }
// LDS index of sequence entry i: one pad entry per 16, which makes the strided stage writes
// (stride 8 and 64 entries) free of bank conflicts
__device__ __forceinline__ int zp(int i) { return i + (i >> 4); }

// Up to N = 2048 the stages alternate between two sequence buffers (one barrier per stage); at
// N = 4096 a second buffer would leave one workgroup per CU, so the stages run in place (two
// barriers per stage).
constexpr bool cfot_two_buffers(int N) { return N <= 2048; }
constexpr int cfot_seq_len(int N) { return N + N / 16; }   // padded sequence, in complex entries

// Dynamic LDS of a cFOT pass: the padded sequence buffer(s) and the stage twiddles.
inline size_t cfot_lds_bytes(int N) {
  return (size_t)(cfot_two_buffers(N) ? 2 : 1) * cfot_seq_len(N) * sizeof(cplx) +
         (size_t)cfot_tw_count(N) * sizeof(cplx);
}
// twiddle table of the dynamic LDS
__device__ __forceinline__ cplx* cfot_lds_tw(cplx* lds, int N) {
  return lds + (cfot_two_buffers(N) ? 2 : 1) * cfot_seq_len(N);
}

// The stage twiddle table of a length-N transform (cfot_tw_count(N) entries).
__global__ void k_cfot_twiddles(int N, cplx* tw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cfot_tw_count(N)) return;
  int NS = 8;
  while (i >= cfot_tw_offset(NS * 8) && NS * 8 < N) NS *= 8;
  const int k = i - cfot_tw_offset(NS);
  const int R = N / NS >= 8 ? 8 : N / NS;
  double s, c;
  sincospi(2.0 * (double)k / (double)(NS * R), &s, &c);
  tw[i] = cplx{c, -s};
}

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * (DIR i)
template <int DIR>
__device__ __forceinline__ cplx cmul_i(cplx a) {
  return DIR > 0 ? cplx{-a.im, a.re} : cplx{a.im, -a.re};
}

// In-register DFT of R = 2, 4 or 8 values, X_q = sum_r v_r exp(DIR 2 pi i r q / R), natural order.
template <int R, int DIR>
__device__ __forceinline__ void dft_small(cplx* v) {
  if constexpr (R == 2) {
    const cplx a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const cplx s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const cplx s13 = cadd(v[1], v[3]), d13 = cmul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  } else {
    static_assert(R == 8, "radix 2, 4 or 8");
    cplx e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft_small<4, DIR>(e);
    dft_small<4, DIR>(o);
    constexpr double h = 0.70710678118654752440;   // exp(DIR 2 pi i q / 8), q = 1, 3
    const cplx w1 = cplx{h, DIR * h}, w3 = cplx{-h, DIR * h};
    const cplx t[4] = {o[0], cmul(o[1], w1), cmul_i<DIR>(o[2]), cmul(o[3], w3)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = cadd(e[q], t[q]);
      v[q + 4] = csub(e[q], t[q]);
    }
  }
}

// One Stockham stage of radix R after sub-transforms of size NS: work item j reads
// zin[j + r N/R], multiplies entry r by w^r with w = exp(DIR 2 pi i (j mod NS) / (NS R)),
// transforms, and writes zout[(j / NS) NS R + (j mod NS) + r NS].  In place (zin == zout) all reads
// finish before the writes.
template <int N, int R, int NS, int DIR, bool INPLACE>
__device__ __forceinline__ void stockham_stage(const cplx* zin, cplx* zout, const cplx* tws) {
  constexpr int T = N / R;                           // work items
  constexpr int IPT = (T + CFOT_THREADS - 1) / CFOT_THREADS;
  cplx v[IPT][R];
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int j = threadIdx.x + it * CFOT_THREADS;
    if (T % CFOT_THREADS == 0 || j < T) {
      const int k = j & (NS - 1);
      cplx w = cplx{1.0, 0.0};
      if constexpr (NS > 1) {
        w = tws[cfot_tw_offset(NS) + k];
        if (DIR > 0) w.im = -w.im;
      }
      cplx wr = w;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const cplx x = zin[zp(j + r * T)];
        if (NS == 1 || r == 0) {
          v[it][r] = x;
        } else {
          v[it][r] = cmul(x, wr);
          if (r + 1 < R) wr = cmul(wr, w);
        }
      }
      dft_small<R, DIR>(v[it]);
    }
  }
  if constexpr (INPLACE) __syncthreads();
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int j = threadIdx.x + it * CFOT_THREADS;
    if (T % CFOT_THREADS == 0 || j < T) {
      const int k = j & (NS - 1);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) zout[zp(base + r * NS)] = v[it][r];
    }
  }
  __syncthreads();
}

// FFT of length N in LDS, natural order in and out (DIR = -1 forward; +1 inverse without 1/N).
// The input is in a; returns the buffer that holds the result (a or b; b is unused when the
// stages run in place).
template <int N, int DIR, int NS = 1>
__device__ __forceinline__ cplx* fft_lds(cplx* a, cplx* b, const cplx* tw) {
  if constexpr (NS < N) {
    constexpr int R = (N / NS) >= 8 ? 8 : N / NS;
    if constexpr (cfot_two_buffers(N)) {
      stockham_stage<N, R, NS, DIR, false>(a, b, tw);
      return fft_lds<N, DIR, NS * R>(b, a, tw);
    } else {
      stockham_stage<N, R, NS, DIR, true>(a, a, tw);
      return fft_lds<N, DIR, NS * R>(a, b, tw);
    }
  } else {
    return a;
  }
}

__device__ __forceinline__ void cfot_load_twiddles(cplx* tw_s, const cplx* tw, int N) {
  for (int k = threadIdx.x; k < cfot_tw_count(N); k += blockDim.x) tw_s[k] = tw[k];
}

// The transform of lambda's circular extension, lambda_c[i] = lambda(i) for i < n and
// lambda_c[N - i] = lambda(i) for 0 < i < n (zero between).  It is real (lambda_c is real and
// even); the rounding residue of its imaginary part is dropped.  One workgroup.
template <int N>
__global__ __launch_bounds__(CFOT_THREADS) void k_cfot_lamhat(int n, double inv_eps, const cplx* tw,
                                                              double* lamhat) {
  extern __shared__ cplx cf_lds[];
  cplx* z = cf_lds;
  cplx* z2 = cf_lds + cfot_seq_len(N);
  cplx* tw_s = cfot_lds_tw(cf_lds, N);
  cfot_load_twiddles(tw_s, tw, N);
  const double s = inv_eps / (2.0 * (double)n * (double)n);
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int d = i < n ? i : (i > N - n ? N - i : -1);
    z[zp(i)] = cplx{d >= 0 ? exp(-(double)d * (double)d * s) : 0.0, 0.0};
  }
  __syncthreads();
  const cplx* r = fft_lds<N, -1>(z, z2, tw_s);
  for (int i = threadIdx.x; i < N; i += blockDim.x) lamhat[i] = r[zp(i)].re;
}

// Row maxima of two rows at once (a in .re, b in .im) over the first n entries.
__device__ __forceinline__ void block_max2(double& a, double& b, double* scratch /* >= 8 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a = fmax(a, __shfl_xor(a, off, 64));
    b = fmax(b, __shfl_xor(b, off, 64));
  }
  __syncthreads();
  if (lane == 0) {
    scratch[2 * wave] = a;
    scratch[2 * wave + 1] = b;
  }
  __syncthreads();
  a = b = -INFINITY;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    a = fmax(a, scratch[2 * w]);
    b = fmax(b, scratch[2 * w + 1]);
  }
}

// Row pair of this workgroup.  Workgroups are dealt to the 8 XCDs round-robin; giving each XCD a
// contiguous range of pairs makes the transposed 16-byte stores of neighbouring pairs (which fill
// the same 128-byte lines) meet in one L2.
__device__ __forceinline__ int cfot_pair() {
  const int nb = gridDim.x, b = blockIdx.x;
  if (nb % 8) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

// Shared body of both passes: rows r0 = 2 cfot_pair() and r0 + 1 of X (log values times
// `scale`, row pitch np, batch stride sX), convolved with lambda, in the dynamic LDS `lds`; returns
// the buffer whose entry zp(k) holds the convolution of row r0 (.re) and row r0 + 1 (.im) times
// N, and sets ma, mb to the row shifts (-inf for a row without mass).
template <int N>
__device__ __forceinline__ const cplx* cfot_convolve_pair(const double* X, double scale, int n, int np,
                                                          const cplx* tw, const double* lamhat, cplx* lds,
                                                          double* scratch, double& ma, double& mb) {
  cplx* z = lds;
  cplx* z2 = lds + cfot_seq_len(N);
  cplx* tw_s = cfot_lds_tw(lds, N);
  static_assert(N % CFOT_THREADS == 0, "whole sequence entries per thread");
  constexpr int PT = N / 2 / CFOT_THREADS > 0 ? N / 2 / CFOT_THREADS : 1;   // row values per thread (n <= N/2)
  constexpr int LT = N / CFOT_THREADS;                                      // sequence entries per thread
  const int tid = threadIdx.x;
  const int r0 = 2 * cfot_pair(), r1 = r0 + 1;
  const bool has1 = r1 < n;
  const double* xa = X + (size_t)r0 * np;
  const double* xb = X + (size_t)r1 * np;
  // every global read first (the rows once, into registers; lambda's transform; the twiddles)
  double ra[PT], rb[PT], lh[LT];
#pragma unroll
  for (int q = 0; q < PT; ++q) {
    const int i = tid + q * CFOT_THREADS;
    ra[q] = i < n ? xa[i] * scale : -INFINITY;
    rb[q] = (i < n && has1) ? xb[i] * scale : -INFINITY;
  }
#pragma unroll
  for (int q = 0; q < LT; ++q) lh[q] = lamhat[tid + q * CFOT_THREADS];
  cfot_load_twiddles(tw_s, tw, N);
  double a = -INFINITY, b = -INFINITY;
#pragma unroll
  for (int q = 0; q < PT; ++q) {
    a = fmax(a, ra[q]);
    b = fmax(b, rb[q]);
  }
  block_max2(a, b, scratch);
  // The shifts returned are the row maxima themselves, -inf for a row without mass: the two rows
  // share one complex transform, whose rounding leaks about 1e-16 of one row into the other, so
  // an empty row's output is not exactly zero; its -inf shift keeps every output of it at -inf.
  ma = a;
  mb = b;
  const double sa = (a > -INFINITY) ? a : 0.0, sb = (b > -INFINITY) ? b : 0.0;
#pragma unroll
  for (int q = 0; q < LT; ++q) {
    const double va = q < PT ? exp(ra[q] - sa) : 0.0;   // entries from N/2 on are padding
    const double vb = q < PT ? exp(rb[q] - sb) : 0.0;
    z[zp(tid + q * CFOT_THREADS)] = cplx{va, vb};
  }
  __syncthreads();
  cplx* zf = fft_lds<N, -1>(z, z2, tw_s);
#pragma unroll
  for (int q = 0; q < LT; ++q) {
    const int i = zp(tid + q * CFOT_THREADS);
    zf[i] = cplx{zf[i].re * lh[q], zf[i].im * lh[q]};
  }
  __syncthreads();
  return fft_lds<N, 1>(zf, zf == z ? z2 : z, tw_s);
}

// m + ln y, -inf for y <= 0 (lost to rounding) or m = -inf (a row without mass)
__device__ __forceinline__ double cfot_log(double y, double m) { return y > 0.0 ? m + log(y) : -INFINITY; }

// Pass 1: outT[k][r] = ln of the row-r convolution at k (rows r of P scaled by 1/eps).  If
// pend_parts is set, workgroup 0 of each target also sums the previous pass 2's marginal-error
// partials (pend_cnt per target, fixed order) into pend_out[target].
// Grid (ceil(n/2), batch), CFOT_THREADS threads, cfot_lds_bytes(N) dynamic LDS.
template <int N>
__global__ __launch_bounds__(CFOT_THREADS) void k_cfot_pass1(const double* P, long long sP, double inv_eps, int n,
                                                             int np, const cplx* tw, const double* lamhat,
                                                             double* outT, long long sO, const double* pend_parts,
                                                             int pend_cnt, double* pend_out) {
  extern __shared__ cplx cf_lds[];
  __shared__ double scratch[8];
  const int bz = blockIdx.y;
  // pending partials, read now so that their latency hides behind the transforms
  const bool pend = pend_parts != nullptr && blockIdx.x == 0;
  double pv = 0.0;
  if (pend)
    for (int i = threadIdx.x; i < pend_cnt; i += CFOT_THREADS) pv += pend_parts[(size_t)bz * pend_cnt + i];
  double ma, mb;
  const cplx* z = cfot_convolve_pair<N>(P + (size_t)bz * sP, inv_eps, n, np, tw, lamhat, cf_lds, scratch, ma, mb);
  const int r0 = 2 * cfot_pair();
  const bool has1 = r0 + 1 < n;
  const double invN = 1.0 / (double)N;
  double* o = outT + (size_t)bz * sO + r0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const cplx y = z[zp(k)];
    o[(size_t)k * np] = cfot_log(y.re * invN, ma);
    if (has1) o[(size_t)k * np + 1] = cfot_log(y.im * invN, mb);
  }
  if (pend) {
    pv = block_sum(pv, scratch);
    if (threadIdx.x == 0) pend_out[bz] = pv;
  }
}

// Pass 2: rows r of Yt convolved again give ln S in row r; the potential update
// Pout[r][j] = eps (lnm[r][j] - ln S) (Eq. 7 or 8 in the log domain), the marginal-error
// partial of the entering plan (same identity as the GEMM path's), the non-finite flag and,
// if requested, ln S itself.  Arrays in the orientation of Pout; one partial per workgroup.
template <int N>
__global__ __launch_bounds__(CFOT_THREADS) void k_cfot_pass2(const double* Yt, long long sY, int n, int np,
                                                             const cplx* tw, const double* lamhat,
                                                             const double* lnm, long long sMarg, double* pot,
                                                             long long sP, double* lnS_out, double eps,
                                                             double* partials, int* flag, int err_on) {
  extern __shared__ cplx cf_lds[];
  __shared__ double scratch[8];
  const int bz = blockIdx.y;
  const int r0 = 2 * cfot_pair();
  constexpr int PT = N / 2 / CFOT_THREADS > 0 ? N / 2 / CFOT_THREADS : 1;
  // the epilogue's inputs, read before the transforms so that their latency is hidden
  double la_v[2][PT], fo_v[2][PT];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int r = r0 + q, j = threadIdx.x + t * CFOT_THREADS;
      const bool ok = r < n && j < n;
      la_v[q][t] = ok ? lnm[(size_t)bz * sMarg + (size_t)r * np + j] : 0.0;
      fo_v[q][t] = (ok && err_on) ? pot[(size_t)bz * sP + (size_t)r * np + j] : 0.0;
    }
  double ma, mb;
  const cplx* z = cfot_convolve_pair<N>(Yt + (size_t)bz * sY, 1.0, n, np, tw, lamhat, cf_lds, scratch, ma, mb);
  const double invN = 1.0 / (double)N, inv_eps = 1.0 / eps;
  double err = 0.0;
  bool bad = false;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = r0 + q;
    if (r >= n) break;
    const double m = q == 0 ? ma : mb;
    double* po = pot + (size_t)bz * sP + (size_t)r * np;
    double* ls = lnS_out ? lnS_out + (size_t)bz * sP + (size_t)r * np : nullptr;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int j = threadIdx.x + t * CFOT_THREADS;
      if (j >= n) break;
      const double y = (q == 0 ? z[zp(j)].re : z[zp(j)].im) * invN;
      const double lnS = cfot_log(y, m);
      const double la = la_v[q][t];
      const bool zm = la == -INFINITY;
      const double fnew = zm ? -INFINITY : eps * (la - lnS);
      if (err_on) {
        const double fold = fo_v[q][t];
        const float tz = exp_err((float)fma(fold, inv_eps, lnS));
        const double d = (fold - fnew) * inv_eps;
        const float df = (float)d, laf = (float)la;
        const float av = exp_err(laf);
        const float ta = (df < 10.0f) ? av * fabsf(expm1_err(df)) : exp_err(laf + df) - av;
        err += (double)(zm ? tz : ta);
      }
      bad = bad || (!zm && !(fabs(fnew) < INFINITY));
      po[j] = fnew;
      if (ls) ls[j] = lnS;
    }
  }
  if (bad) atomicOr(flag, 1);
  if (err_on) {
    err = block_sum(err, scratch);
    if (threadIdx.x == 0) partials[(size_t)bz * gridDim.x + blockIdx.x] = err;
  }
}

// out[b] = sum of parts[b][0 .. cnt) in a fixed order (one workgroup per target).
__global__ void k_cfot_sum(const double* parts, int cnt, double* out) {
  __shared__ double red[4];
  const int bz = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) s += parts[(size_t)bz * cnt + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[bz] = s;
}

// out[b][c][r] = in[b][r][c] for r, c < n (row pitch np); 32 x 32 tiles through LDS.
__global__ void k_transpose64(const double* in, long long sIn, double* out, long long sOut, int n, int np) {
  __shared__ double t[32][33];
  const int bz = blockIdx.z;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 8 rows per pass
  const double* src = in + (size_t)bz * sIn;
  double* dst = out + (size_t)bz * sOut;
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + y, c = c0 + tx;
    t[y][tx] = (r < n && c < n) ? src[(size_t)r * np + c] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int c = c0 + y, r = r0 + tx;
    if (r < n && c < n) dst[(size_t)c * np + r] = t[tx][y];
  }
}

}  // namespace fot
