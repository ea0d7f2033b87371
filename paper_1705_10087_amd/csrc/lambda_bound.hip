// Window energies of the signal for the error bound of the split-bf16
// correlation (MIXED policy): lambda_max = max |D^T X| (eq. (2): the smallest
// lambda with Z = 0 optimal) is taken from the split-bf16 values only after
// every entry that the rounding error could make the maximum is recomputed in
// double.  The error of one entry beta_k[t] is at most
// c sum_{p,tau} |D_k[p][tau]| |X[p][t + tau]| <= c |D_k| |X[., t : t + W]|
// (Cauchy-Schwarz), so the host needs max_t |X[., t : t + W]|^2 per signal.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dicod_internal.h"

namespace dicod {
namespace {

constexpr int kEnergyTile = 256;  // positions t per workgroup (the kTile tiling)

// out_bits[sig] = max over t in the tile of sum_p sum_{tau < W} X[p][t + tau]^2,
// as the bit pattern of a non-negative double (atomic max on the bits).
__global__ void __launch_bounds__(256)
k_win_energy_max(const float* __restrict__ X, int P, int W, const SigDesc* __restrict__ sig,
                 const int64_t* __restrict__ tile_pref, int n_sig,
                 unsigned long long* __restrict__ out_bits)
{
    extern __shared__ double q[];  // [kEnergyTile + W - 1] channel sums of squares
    const int64_t tile = blockIdx.x;
    int lo = 0, hi = n_sig - 1;  // signal of this tile: last si with tile_pref[si] <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (tile_pref[mid] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    const SigDesc sd = sig[lo];
    const int64_t t0 = (tile - tile_pref[lo]) * kEnergyTile;
    const int64_t n = (int64_t)kEnergyTile + W - 1 < sd.T - t0 ? (int64_t)kEnergyTile + W - 1
                                                               : sd.T - t0;
    const float* __restrict__ xs = X + sd.x_off;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double s = 0.0;
        for (int p = 0; p < P; ++p) {
            const double v = (double)xs[(int64_t)p * sd.T + t0 + i];
            s += v * v;
        }
        q[i] = s;
    }
    __syncthreads();
    double m = 0.0;
    const int64_t t = t0 + threadIdx.x;
    if (threadIdx.x < kEnergyTile && t < sd.L) {
        double s = 0.0;
        for (int tau = 0; tau < W; ++tau)
            s += q[threadIdx.x + tau];
        m = s;
    }
    for (int o = 32; o > 0; o >>= 1)
        m = fmax(m, __shfl_xor(m, o));
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        atomicMax(&out_bits[lo], (unsigned long long)__double_as_longlong(m));
    }
}

// thr[i] = max(0, v_i - 2 coef sqrt(e_i)): v_i the largest split-bf16 |beta|
// of signal i, e_i its largest window energy, coef = 1.05 c max_k |D_k| (the
// per-entry error bound above with a 5% margin).  The maximiser's split value
// is at least lambda_max - e >= v - 2 e, so every entry that can be the
// maximum has a split value >= thr.
__global__ void k_refine_threshold(const unsigned long long* __restrict__ vbits,
                                   const unsigned long long* __restrict__ ebits, int n,
                                   double coef, double* __restrict__ thr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double v = __longlong_as_double((long long)vbits[i]);
    const double e = coef * sqrt(__longlong_as_double((long long)ebits[i]));
    const double t = v - 2.0 * e;
    thr[i] = t > 0.0 ? t : 0.0;
}

}  // namespace

hipError_t launch_refine_threshold(const unsigned long long* vbits,
                                   const unsigned long long* ebits, int n, double coef,
                                   double* thr, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_refine_threshold, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       vbits, ebits, n, coef, thr);
    return hipGetLastError();
}

double refine_coef(int P, int W, double dnorm_max)
{
    const double c = 3.1 * std::ldexp(1.0, -16) + ((double)P * W + 1.0) * std::ldexp(1.0, -24);
    return 1.05 * c * dnorm_max;
}

size_t win_energy_lds_bytes(int W) { return ((size_t)kEnergyTile + W - 1) * sizeof(double); }

hipError_t launch_win_energy_max(const float* X, int P, int W, const SigDesc* sig,
                                 const int64_t* tile_pref, int n_sig, int64_t n_tiles,
                                 unsigned long long* out_bits, hipStream_t s)
{
    if (n_tiles <= 0)
        return hipSuccess;
    const size_t lds = win_energy_lds_bytes(W);
    if (lds > kLdsBytes)
        return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)k_win_energy_max,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_win_energy_max, dim3((unsigned)n_tiles), dim3(256), lds, s, X, P, W,
                       sig, tile_pref, n_sig, out_bits);
    return hipGetLastError();
}

}  // namespace dicod
