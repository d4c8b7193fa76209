// Output beam of a phase and Gerchberg-Saxton polishing for gfx950.
//
// The far field of Eq. 1 (arXiv 2512.19072, Sec. 2) is the discrete Fourier transform between
// the two centred grids, F[f]_LM = sum_jk f_jk exp(-2 pi i ((j-c)(L-c) + (k-c)(M-c)) / n) with
// c = floor(n/2) (x_j X_L = (j-c)(L-c)/n in the paper's units).  It is evaluated as two complex
// matrix products F = W f W^T, each as two real MFMA GEMMs (C = A . B^T, FP64) whose K index
// runs over the real and then the imaginary half of a row:
//
//   f    [np][2np]  = [Re f | Im f]              (row j)
//   Wa   [np][2np]  = [Re W | -Im W]             Wb = [Im W | Re W]         (row L)
//   step A  Ht[M][.] = [Re | Im] of sum_k W[M][k] f[j][k]   = (Wa . f^T, Wb . f^T)
//   step B  F[L][.]  = [Re | Im] of sum_j W[L][j] Ht[M][j]  = (Wa . Ht^T, Wb . Ht^T)
//
// The inverse transform (up to 1/n^2) uses conj(W): Wca = [Re W | Im W], Wcb = [-Im W | Re W].
// The intensity, the L1 loss of Sec. 4 and the Gerchberg-Saxton projections are elementwise
// kernels around these products.  Padded rows and columns of every operand are zero.
#pragma once

#include "fot_kernels.hpp"

namespace fot {

// The four K-concatenated DFT operands, [np][2np] each.  The integer phase (L-c)(j-c) is
// reduced mod n before the FP64 sincospi, so every entry is a root of unity to FP64 rounding.
__global__ void k_dft_operands(int n, int np, double* Wa, double* Wb, double* Wca, double* Wcb) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  const int L = (int)(idx / np), j = (int)(idx % np);
  double re = 0.0, im = 0.0;
  if (L < n && j < n) {
    const long long c = n / 2;
    long long r = ((long long)(L - c) * (long long)(j - c)) % n;
    if (r < 0) r += n;
    double s, co;
    sincospi(2.0 * (double)r / (double)n, &s, &co);
    re = co;
    im = -s;   // exp(-2 pi i r / n)
  }
  const size_t row = (size_t)L * 2 * np;
  Wa[row + j] = re;
  Wa[row + np + j] = -im;
  Wb[row + j] = im;
  Wb[row + np + j] = re;
  Wca[row + j] = re;
  Wca[row + np + j] = im;
  Wcb[row + j] = -im;
  Wcb[row + np + j] = re;
}

// f = g e^{2 pi i phi} into the [Re | Im] row layout; one block per row j, grid (n, batch).
// g is [n][n] (shared by the batch), phi [batch][n][n].
__global__ void k_beam_field(const double* g, const double* phase, int n, int np, double* fc) {
  const int j = blockIdx.x, bz = blockIdx.y;
  const double* ph = phase + ((size_t)bz * n + j) * n;
  double* out = fc + ((size_t)bz * np + j) * 2 * np;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double v = g[(size_t)j * n + k];
    double s, co;
    sincospi(2.0 * ph[k], &s, &co);
    out[k] = v * co;
    out[np + k] = v * s;
  }
}

// Unit-power intensity I = |F|^2 * inv_power[b] (inv_power = 1 / (n^2 sum g^2), Parseval) and,
// if G is given, the row sums of |I - G^2 / sum G^2| (sumG2[b]).  One block per row L.
__global__ void k_beam_intensity(const double* F, int n, int np, const double* inv_power, const double* G,
                                 const double* sumG2, double* I_out, double* rowpart) {
  __shared__ double red[4];
  const int L = blockIdx.x, bz = blockIdx.y;
  const double* Fr = F + ((size_t)bz * np + L) * 2 * np;
  const double scale = inv_power[bz];
  const double inv_b = G ? 1.0 / sumG2[bz] : 0.0;
  double s = 0.0;
  for (int M = threadIdx.x; M < n; M += blockDim.x) {
    const double re = Fr[M], im = Fr[np + M];
    const double I = (re * re + im * im) * scale;
    if (I_out) I_out[((size_t)bz * n + L) * n + M] = I;
    if (G) {
      const double t = G[((size_t)bz * n + L) * n + M];
      s += fabs(I - t * t * inv_b);
    }
  }
  s = block_sum(s, red);
  if (G && threadIdx.x == 0) rowpart[(size_t)bz * n + L] = s;
}

// out[b] = sum of rows[b][0 .. n) in a fixed order; one block per b.
__global__ void k_sum_rows(const double* rows, int n, double* out) {
  __shared__ double red[4];
  const int bz = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += rows[(size_t)bz * n + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[bz] = s;
}

// 1 / (n^2 sum g^2) for every target from the row sums of g^2 (the same g for the batch).
__global__ void k_inv_power(const double* rowsum_g, int n, int batch, double* inv_power) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += rowsum_g[i];
  s = block_sum(s, red);
  for (int b = threadIdx.x; b < batch; b += blockDim.x) inv_power[b] = 1.0 / ((double)n * (double)n * s);
}

// Fourier-plane projection of Gerchberg-Saxton: F <- G F / |F| (G where F = 0), written into the
// [Re | Im] operand layout of the inverse transform.  One block per row L.
__global__ void k_gs_project(const double* F, const double* G, int n, int np, double* fc) {
  const int L = blockIdx.x, bz = blockIdx.y;
  const double* Fr = F + ((size_t)bz * np + L) * 2 * np;
  double* out = fc + ((size_t)bz * np + L) * 2 * np;
  for (int M = threadIdx.x; M < n; M += blockDim.x) {
    const double re = Fr[M], im = Fr[np + M];
    const double mag = hypot(re, im);
    const double t = G[((size_t)bz * n + L) * n + M];
    out[M] = mag > 0.0 ? t * (re / mag) : t;
    out[np + M] = mag > 0.0 ? t * (im / mag) : 0.0;
  }
}

// Input-plane projection: phi = arg(f) / (2 pi) in (-1/2, 1/2] (0 where f = 0) and the next
// field g e^{2 pi i phi} = g f / |f|.  One block per row j.
__global__ void k_gs_phase(const double* F, const double* g, int n, int np, double* phase, double* fc) {
  const int j = blockIdx.x, bz = blockIdx.y;
  const double* fr = F + ((size_t)bz * np + j) * 2 * np;
  double* out = fc + ((size_t)bz * np + j) * 2 * np;
  double* ph = phase + ((size_t)bz * n + j) * n;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double re = fr[k], im = fr[np + k];
    const double mag = hypot(re, im);
    const double v = g[(size_t)j * n + k];
    ph[k] = atan2(im, re) * (0.5 / M_PI);
    out[k] = mag > 0.0 ? v * (re / mag) : v;
    out[np + k] = mag > 0.0 ? v * (im / mag) : 0.0;
  }
}

}  // namespace fot
