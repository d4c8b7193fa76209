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
// LDS: a radix-2 decimation-in-frequency forward FFT (natural order in, bit-reversed out), the
// product with lambda's transform held in the same bit-reversed order, and a radix-2
// decimation-in-time inverse (bit-reversed in, natural out), so no permutation pass is needed.
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
constexpr int CFOT_MAX_N = 4096;   // FFT length limit (n <= 2048)

// Dynamic LDS of a cFOT pass: the sequence (N complex) and the twiddles (N/2 complex).
inline size_t cfot_lds_bytes(int N) { return (size_t)N * sizeof(cplx) + (size_t)(N / 2) * sizeof(cplx); }

// tw[k] = exp(-2 pi i k / N), k < N/2
__global__ void k_cfot_twiddles(int N, cplx* tw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N / 2) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)N, &s, &c);
  tw[k] = cplx{c, -s};
}

// Forward FFT in place, natural order in, bit-reversed order out (radix-2, decimation in frequency).
__device__ __forceinline__ void fft_dif(cplx* z, const cplx* tw, int N) {
  for (int m = N; m >= 2; m >>= 1) {
    const int half = m >> 1, ts = N / m;
    const int lh = __builtin_ctz(half);
    for (int q = threadIdx.x; q < N / 2; q += blockDim.x) {
      const int g = q >> lh, j = q & (half - 1);
      const int i0 = g * m + j, i1 = i0 + half;
      const cplx a = z[i0], b = z[i1], w = tw[j * ts];
      z[i0] = cplx{a.re + b.re, a.im + b.im};
      const double dr = a.re - b.re, di = a.im - b.im;
      z[i1] = cplx{dr * w.re - di * w.im, dr * w.im + di * w.re};
    }
    __syncthreads();
  }
}

// Inverse FFT in place without the 1/N, bit-reversed order in, natural order out (radix-2,
// decimation in time, conjugate twiddles).
__device__ __forceinline__ void fft_dit_inv(cplx* z, const cplx* tw, int N) {
  for (int m = 2; m <= N; m <<= 1) {
    const int half = m >> 1, ts = N / m;
    const int lh = __builtin_ctz(half);
    for (int q = threadIdx.x; q < N / 2; q += blockDim.x) {
      const int g = q >> lh, j = q & (half - 1);
      const int i0 = g * m + j, i1 = i0 + half;
      const cplx a = z[i0], c = z[i1], w = tw[j * ts];
      // b = c * conj(w)
      const double br = c.re * w.re + c.im * w.im, bi = c.im * w.re - c.re * w.im;
      z[i0] = cplx{a.re + br, a.im + bi};
      z[i1] = cplx{a.re - br, a.im - bi};
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void cfot_load_twiddles(cplx* tw_s, const cplx* tw, int N) {
  for (int k = threadIdx.x; k < N / 2; k += blockDim.x) tw_s[k] = tw[k];
}

// The transform of lambda's circular extension, lambda_c[i] = lambda(i) for i < n and
// lambda_c[N - i] = lambda(i) for 0 < i < n (zero between), in the bit-reversed order of
// fft_dif.  It is real (lambda_c is real and even); the rounding residue of its imaginary part
// is dropped.  One workgroup.
__global__ __launch_bounds__(CFOT_THREADS) void k_cfot_lamhat(int n, int N, double inv_eps, const cplx* tw,
                                                              double* lamhat) {
  extern __shared__ cplx cf_lds[];
  cplx* z = cf_lds;
  cplx* tw_s = cf_lds + N;
  cfot_load_twiddles(tw_s, tw, N);
  const double s = inv_eps / (2.0 * (double)n * (double)n);
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int d = i < n ? i : (i > N - n ? N - i : -1);
    z[i] = cplx{d >= 0 ? exp(-(double)d * (double)d * s) : 0.0, 0.0};
  }
  __syncthreads();
  fft_dif(z, tw_s, N);
  for (int i = threadIdx.x; i < N; i += blockDim.x) lamhat[i] = z[i].re;
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

// Shared body of both passes: rows r0 = 2 blockIdx.x and r0 + 1 of X (log values times
// `scale`, row pitch np, batch stride sX), convolved with lambda; on return z[k] holds the
// convolution of row r0 (.re) and row r0 + 1 (.im) times N, and ma, mb the row shifts.
__device__ __forceinline__ void cfot_convolve_pair(const double* X, double scale, int n, int np, int N,
                                                   const cplx* tw, const double* lamhat, cplx* z, cplx* tw_s,
                                                   double* scratch, double& ma, double& mb) {
  const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
  const bool has1 = r1 < n;
  const double* xa = X + (size_t)r0 * np;
  const double* xb = X + (size_t)r1 * np;
  cfot_load_twiddles(tw_s, tw, N);
  double a = -INFINITY, b = -INFINITY;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a = fmax(a, xa[i] * scale);
    if (has1) b = fmax(b, xb[i] * scale);
  }
  block_max2(a, b, scratch);
  ma = (a > -INFINITY) ? a : 0.0;   // an all-zero row stays zero
  mb = (b > -INFINITY) ? b : 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const bool ok = i < n;
    const double va = ok ? exp(xa[i] * scale - ma) : 0.0;
    const double vb = (ok && has1) ? exp(xb[i] * scale - mb) : 0.0;
    z[i] = cplx{va, vb};
  }
  __syncthreads();
  fft_dif(z, tw_s, N);
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const double l = lamhat[i];
    z[i] = cplx{z[i].re * l, z[i].im * l};
  }
  __syncthreads();
  fft_dit_inv(z, tw_s, N);
}

__device__ __forceinline__ double cfot_log(double y, double m) { return y > 0.0 ? m + log(y) : -INFINITY; }

// Pass 1: outT[k][r] = ln of the row-r convolution at k (rows r of P scaled by 1/eps).
// Grid (ceil(n/2), batch), CFOT_THREADS threads, cfot_lds_bytes(N) dynamic LDS.
__global__ __launch_bounds__(CFOT_THREADS) void k_cfot_pass1(const double* P, long long sP, double inv_eps, int n,
                                                             int np, int N, const cplx* tw, const double* lamhat,
                                                             double* outT, long long sO) {
  extern __shared__ cplx cf_lds[];
  __shared__ double scratch[8];
  cplx* z = cf_lds;
  cplx* tw_s = cf_lds + N;
  const int bz = blockIdx.y;
  double ma, mb;
  cfot_convolve_pair(P + (size_t)bz * sP, inv_eps, n, np, N, tw, lamhat, z, tw_s, scratch, ma, mb);
  const int r0 = 2 * blockIdx.x;
  const bool has1 = r0 + 1 < n;
  const double invN = 1.0 / (double)N;
  double* o = outT + (size_t)bz * sO + r0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const cplx y = z[k];
    o[(size_t)k * np] = cfot_log(y.re * invN, ma);
    if (has1) o[(size_t)k * np + 1] = cfot_log(y.im * invN, mb);
  }
}

// Pass 2: rows r of Yt convolved again give ln S in row r; the potential update
// Pout[r][j] = eps (lnm[r][j] - ln S) (Eq. 7 or 8 in the log domain), the marginal-error
// partial of the entering plan (same identity as the GEMM path's), the non-finite flag and,
// if requested, ln S itself.  Arrays in the orientation of Pout; one partial per workgroup.
__global__ __launch_bounds__(CFOT_THREADS) void k_cfot_pass2(const double* Yt, long long sY, int n, int np, int N,
                                                             const cplx* tw, const double* lamhat,
                                                             const double* lnm, long long sMarg, double* pot,
                                                             long long sP, double* lnS_out, double eps,
                                                             double* partials, int* flag, int err_on) {
  extern __shared__ cplx cf_lds[];
  __shared__ double scratch[8];
  cplx* z = cf_lds;
  cplx* tw_s = cf_lds + N;
  const int bz = blockIdx.y;
  double ma, mb;
  cfot_convolve_pair(Yt + (size_t)bz * sY, 1.0, n, np, N, tw, lamhat, z, tw_s, scratch, ma, mb);
  const int r0 = 2 * blockIdx.x;
  const double invN = 1.0 / (double)N, inv_eps = 1.0 / eps;
  double err = 0.0;
  bool bad = false;
  for (int q = 0; q < 2; ++q) {
    const int r = r0 + q;
    if (r >= n) break;
    const double m = q == 0 ? ma : mb;
    const double* lm = lnm + (size_t)bz * sMarg + (size_t)r * np;
    double* po = pot + (size_t)bz * sP + (size_t)r * np;
    double* ls = lnS_out ? lnS_out + (size_t)bz * sP + (size_t)r * np : nullptr;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const double y = (q == 0 ? z[j].re : z[j].im) * invN;
      const double lnS = cfot_log(y, m);
      const double la = lm[j];
      const bool zm = la == -INFINITY;
      const double fnew = zm ? -INFINITY : eps * (la - lnS);
      if (err_on) {
        const double fold = po[j];
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
