// The field-like DAS sampling K_r of eq.(3) on recorded point strains e[nch][nt] (x-x
// strain at each channel's normal node at t_{n+1}, channels in fiber order): the mean over
// a gauge of consecutive channels, optionally the strain rate (first difference in time at
// the simulation step, e(t_0) = 0) and a resampling to every decim-th sample (those at
// t_{n+1} = k decim dt). Field data are [nch - gauge + 1][nt / decim]. The misfit's
// transpose enters the transposed sweep through the reverse cumulative sum of the
// residual, so K^T is applied in that form: with the strain rate the cumulative sum of the
// time difference's transpose telescopes, and e_bar is the resampled residual's gauge
// spread over dt.
#include <algorithm>

#include "efwi_internal.h"

namespace efwi {
namespace {

constexpr int RB_ = 128;

// Field sample (f, k) of K e, in FP64: the gauge's channels summed in order, then scaled.
__device__ __forceinline__ double field_sample(const Receiver& R, const float* __restrict__ e, int f, int k) {
  const int n = k * R.decim + R.decim - 1;
  double s = 0.0;
  for (int c = f; c < f + R.gauge; ++c) {
    const float* row = e + (long)c * R.nt;
    double x = row[n];
    if (R.rate) x = (x - (n > 0 ? (double)row[n - 1] : 0.0)) * (double)R.rdt;
    s += x;
  }
  return s * (1.0 / R.gauge);
}

// One thread per field sample (consecutive threads take consecutive times of a channel).
__global__ __launch_bounds__(RB_) void k_field_data(Receiver R, const float* __restrict__ e, float* __restrict__ out,
                                                    long total) {
  const int ntf = R.nt / R.decim;
  for (long q = blockIdx.x * (long)RB_ + threadIdx.x; q < total; q += (long)gridDim.x * RB_) {
    const int f = (int)(q / ntf), k = (int)(q - (long)f * ntf);
    out[q] = (float)field_sample(R, e, f, k);
  }
}

// One thread per field channel f: the residual K e - dobs at every resampled time into rf
// and the FP64 sum of its squares into partial[f].
__global__ __launch_bounds__(RB_) void k_field_residual(Receiver R, const float* __restrict__ e,
                                                        const float* __restrict__ dobs, float* __restrict__ rf,
                                                        double* __restrict__ partial) {
  const int f = blockIdx.x * RB_ + threadIdx.x;
  const int nf = R.nch - R.gauge + 1, ntf = R.nt / R.decim;
  if (f >= nf) return;
  double sq = 0.0;
  for (int k = 0; k < ntf; ++k) {
    const long o = (long)f * ntf + k;
    const double r = field_sample(R, e, f, k) - (double)dobs[o];
    sq += r * r;
    rf[o] = (float)r;
  }
  partial[f] = sq;
}

__global__ __launch_bounds__(256) void k_field_phi(const double* __restrict__ partial, int n,
                                                   double* __restrict__ phi) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) a += partial[k];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *phi = 0.5 * sh[0];
}

// One thread per recorded channel c: e_bar[n][c] = sum_{k >= n} (K^T rf)[c][k], written for
// every n (descending).
__global__ __launch_bounds__(RB_) void k_field_ebar(Receiver R, const float* __restrict__ rf,
                                                    float* __restrict__ ebar) {
  const int c = blockIdx.x * RB_ + threadIdx.x;
  if (c >= R.nch) return;
  const int nf = R.nch - R.gauge + 1, ntf = R.nt / R.decim;
  const int f0 = std::max(0, c - R.gauge + 1), f1 = std::min(c, nf - 1);
  const double inv_g = 1.0 / R.gauge;
  double cum = 0.0;
  for (int n = R.nt - 1; n >= 0; --n) {
    double y = 0.0;
    const int k = n / R.decim;
    if (n - k * R.decim == R.decim - 1 && k < ntf)
      for (int f = f0; f <= f1; ++f) y += (double)rf[(long)f * ntf + k];
    double v;
    if (R.rate) {
      v = y * (double)R.rdt * inv_g;
    } else {
      cum += y;
      v = cum * inv_g;
    }
    ebar[(long)n * R.nch + c] = (float)v;
  }
}

int blocks(int n) { return std::max(1, (n + RB_ - 1) / RB_); }

// Field channels actually formed: none without recorded channels.
int field_rows(const Receiver& R) { return R.nch > 0 ? std::max(0, R.nch - R.gauge + 1) : 0; }

}  // namespace

hipError_t launch_field_data(const Receiver& R, const float* e, float* out, hipStream_t st) {
  const long total = (long)field_rows(R) * (R.nt / R.decim);
  if (total > 0) {
    const long nb = std::min<long>((total + RB_ - 1) / RB_, 4096);
    k_field_data<<<(int)nb, RB_, 0, st>>>(R, e, out, total);
  }
  return hipGetLastError();
}

hipError_t launch_field_misfit(const Receiver& R, const float* e, const float* dobs, float* rf, double* partial,
                               double* phi, float* ebar, hipStream_t st) {
  const int nf = field_rows(R);
  if (nf > 0) k_field_residual<<<blocks(nf), RB_, 0, st>>>(R, e, dobs, rf, partial);
  k_field_phi<<<1, 256, 0, st>>>(partial, nf, phi);
  if (R.nch > 0) k_field_ebar<<<blocks(R.nch), RB_, 0, st>>>(R, rf, ebar);
  return hipGetLastError();
}

hipError_t launch_field_cumsum(const Receiver& R, const float* rf, float* ebar, hipStream_t st) {
  if (R.nch > 0) k_field_ebar<<<blocks(R.nch), RB_, 0, st>>>(R, rf, ebar);
  return hipGetLastError();
}

}  // namespace efwi
