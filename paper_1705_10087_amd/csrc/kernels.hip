// gfx950 kernels for locally greedy convolutional coordinate descent.
//
// Notation follows Moreau, Oudre & Vayatis (ICML 2018): X [P][T], atoms
// D [K][P][W], activations Z [K][L] with L = T - W + 1, the auxiliary
// variable beta of Sec. 2.1 and the correlation table S of eq. (3).
//
// The descent keeps g = beta - |D_k|^2 Z instead of beta (g is the
// correlation of D_k with the full residual).  With g the update of eq. (3)
// applies uniformly, including at the updated coordinate, and g stays of the
// order of lambda near the solution, which keeps single precision usable.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>
#include <utility>

#include "dicod_internal.h"

namespace dicod {

typedef double d4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1, so that register
// arrays indexed by i are never indexed dynamically.
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Largest i with pref[i] <= x (pref has n + 1 non-decreasing entries).
__device__ __forceinline__ int find_sig(const int64_t* __restrict__ pref, int n,
                                        int64_t x)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, T v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

template <typename T>
static hipError_t fill(T* p, T v, size_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s)
{
    return fill<uint32_t>(p, v, n, s);
}
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, size_t n,
                           hipStream_t s)
{
    return fill<unsigned long long>(p, v, n, s);
}
hipError_t launch_fill_f64(double* p, double v, size_t n, hipStream_t s)
{
    return fill<double>(p, v, n, s);
}

// ---------------------------------------------------------------------------
// Correlation out_k[t] = sum_{p,tau} D_k[p][tau] Y[p][t + tau] on f64 MFMA.
//
// Implicit im2col: the GEMM is [K x PW] . [PW x L]; a workgroup owns 256
// output positions and 32 atoms, stages its Y window [P][256 + W - 1] in LDS
// once and walks the reduction index r = p W + tau in chunks of 64, staging the
// matching slice of D.  Each wave computes 32 atoms x 64 positions with
// v_mfma_f64_16x16x4f64 (A = D slice, B = shifted Y rows).
// ---------------------------------------------------------------------------
// Workgroup barrier that orders LDS only: unlike __syncthreads() it does not
// wait for the block's outstanding global loads.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kCorrRCMax = 100;  // staged atom taus per pass, at most
constexpr int kCorrPre = 13;     // staged atom values per thread: 32 x 100 <= 13 x 256

// taus per staged pass: W rounded up to a multiple of 4, split into equal
// passes of at most kCorrRCMax (also multiples of 4)
__host__ __device__ inline int corr_chunk(int W)
{
    const int Wq = (W + 3) & ~3;
    const int n = (Wq + kCorrRCMax - 1) / kCorrRCMax;
    return ((Wq + n - 1) / n + 3) & ~3;
}

template <typename TY>
__global__ void __launch_bounds__(256)
k_corr_f64(const double* __restrict__ D, int K, int P, int W,
           const TY* __restrict__ Y, const SigDesc* __restrict__ sig,
           const int64_t* __restrict__ tile_pref, int n_sig,
           double* __restrict__ out64, float* __restrict__ g32,
           double* __restrict__ g64, double* __restrict__ z0, float* __restrict__ z32_0,
           unsigned long long* __restrict__ amax_bits)
{
    extern __shared__ double lds[];
    const int ystride = kTile + ((W + 3) & ~3);          // window + padded taus
    double* Dc = lds;                                     // [32][corr_chunk + 1]
    double* Ys = lds + 32 * (corr_chunk(W) + 1);          // [P][ystride]

    const int64_t tile = blockIdx.x;
    const int si = find_sig(tile_pref, n_sig, tile);
    const SigDesc sd = sig[si];
    const int64_t t_a = (tile - tile_pref[si]) * kTile;
    const int kbase = blockIdx.y * 32;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    // loads at clamped (valid) indices, unconditional: several in flight
#pragma unroll 4
    for (int i = tid; i < P * ystride; i += 256) {
        const int p = i / ystride;
        const int64_t t = t_a + (i - p * ystride);
        const double y = (double)Y[sd.x_off + (int64_t)p * sd.T + (t < sd.T ? t : sd.T - 1)];
        Ys[i] = t < sd.T ? y : 0.0;
    }

    d4_t acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};

    // the reduction runs channel by channel over tau in chunks of rc (a
    // multiple of 4; taus past W have zero atoms), so a lane's B row needs no
    // index division
    const int arow = lane & 15;
    const int kk = lane >> 4;
    const int Wq = (W + 3) & ~3;
    const int rc = corr_chunk(W);
    const int ds = rc + 1;  // odd stride: no LDS bank aliasing
    // The next pass's atom values are loaded into registers (at clamped, valid
    // indices, all in flight together) while the current pass's products run;
    // the barriers order LDS only, so they do not wait for those loads.
    const int ncp = (Wq + rc - 1) / rc;  // passes per channel
    const int npass = P * ncp;
    double dv[kCorrPre];
    auto load_d = [&](int pass) __attribute__((always_inline)) {
        const int p = pass / ncp;
        const int tau0 = (pass - p * ncp) * rc;
#pragma unroll
        for (int q = 0; q < kCorrPre; ++q) {
            const int i = tid + 256 * q;
            const int m = i / rc;
            const int k = kbase + m < K ? kbase + m : K - 1;
            const int tau = tau0 + (i - m * rc) < W ? tau0 + (i - m * rc) : W - 1;
            dv[q] = D[((int64_t)k * P + p) * W + tau];
        }
    };
    load_d(0);
    for (int pass = 0; pass < npass; ++pass) {
        const int p = pass / ncp;
        const int tau0 = (pass - p * ncp) * rc;
        const int nr = Wq - tau0 < rc ? Wq - tau0 : rc;
        lds_barrier();  // the previous pass's atoms are consumed
#pragma unroll
        for (int q = 0; q < kCorrPre; ++q) {
            const int i = tid + 256 * q;
            if (i < 32 * rc) {
                const int m = i / rc;
                const int rr = i - m * rc;
                Dc[m * ds + rr] = (kbase + m < K && tau0 + rr < W) ? dv[q] : 0.0;
            }
        }
        if (pass + 1 < npass)
            load_d(pass + 1);
        lds_barrier();
        const double* __restrict__ da = Dc + arow * ds + kk;
        const double* __restrict__ yb = Ys + p * ystride + wave * 64 + arow + tau0 + kk;
        for (int ks = 0; ks < nr; ks += 4) {
            const double a0 = da[ks];
            const double a1 = da[16 * ds + ks];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const double bv = yb[ks + nt * 16];
                acc[0][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv, acc[0][nt], 0, 0, 0);
                acc[1][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv, acc[1][nt], 0, 0, 0);
            }
        }
    }

    // C[i][j] of a 16x16 f64 MFMA tile sits in lane (i % 4) * 16 + j, item i / 4
    // (measured on gfx950; the f32/bf16 tiles use lane (i / 4) * 16 + j, item i % 4).
    // Optionally the same pass zeroes the descent's Z (and its float copy) at
    // these coordinates and takes max |beta| (lambda_max, eq. 2) per signal.
    double amax = 0.0;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = kbase + mi * 16 + kk + 4 * v;
                const int64_t t = t_a + wave * 64 + nt * 16 + arow;
                if (k < K && t < sd.L) {
                    const double val = acc[mi][nt][v];
                    const int64_t o = sd.z_off + (int64_t)k * sd.L + t;
                    out64[o] = val;
                    if (g32)
                        g32[o] = (float)val;
                    if (g64)
                        g64[o] = val;
                    if (z0)
                        z0[o] = 0.0;
                    if (z32_0)
                        z32_0[o] = 0.0f;
                    amax = fmax(amax, fabs(val));
                }
            }
    if (amax_bits) {
        for (int o = 32; o > 0; o >>= 1)
            amax = fmax(amax, __shfl_xor(amax, o));
        if ((threadIdx.x & 63) == 0)  // non-negative doubles order as their bits
            atomicMax(&amax_bits[si], (unsigned long long)__double_as_longlong(amax));
    }
}

static size_t corr_lds(int P, int W)
{
    return sizeof(double) * (32 * (size_t)(corr_chunk(W) + 1) + (size_t)P * (kTile + ((W + 3) & ~3)));
}

hipError_t launch_corr_f64_x32(const double* D, int K, int P, int W, const float* Y,
                               const SigDesc* sig, const int64_t* tile_pref,
                               int n_sig, int64_t n_tiles, double* out64,
                               float* g32, double* g64, hipStream_t s, double* z0,
                               float* z32_0, unsigned long long* amax_bits)
{
    size_t lds = corr_lds(P, W);
    if (lds > kLdsBytes)
        return hipErrorInvalidValue;
    (void)hipFuncSetAttribute((const void*)k_corr_f64<float>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (n_tiles <= 0)
        return hipSuccess;
    dim3 grid((unsigned)n_tiles, (unsigned)((K + 31) / 32));
    hipLaunchKernelGGL(k_corr_f64<float>, grid, dim3(256), lds, s, D, K, P, W, Y,
                       sig, tile_pref, n_sig, out64, g32, g64, z0, z32_0, amax_bits);
    return hipGetLastError();
}

hipError_t launch_corr_f64_x64(const double* D, int K, int P, int W,
                               const double* Y, const SigDesc* sig,
                               const int64_t* tile_pref, int n_sig,
                               int64_t n_tiles, double* out64, hipStream_t s)
{
    size_t lds = corr_lds(P, W);
    if (lds > kLdsBytes)
        return hipErrorInvalidValue;
    (void)hipFuncSetAttribute((const void*)k_corr_f64<double>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (n_tiles <= 0)
        return hipSuccess;
    dim3 grid((unsigned)n_tiles, (unsigned)((K + 31) / 32));
    hipLaunchKernelGGL(k_corr_f64<double>, grid, dim3(256), lds, s, D, K, P, W, Y,
                       sig, tile_pref, n_sig, out64, (float*)nullptr,
                       (double*)nullptr, (double*)nullptr, (float*)nullptr,
                       (unsigned long long*)nullptr);
    return hipGetLastError();
}

// Split-bf16 correlation (MIXED policy): every float x is split into
// hi = bf16(x) and lo = bf16(x - hi), and hi*hi + hi*lo + lo*hi accumulate in
// fp32 on v_mfma_f32_16x16x32_bf16 (lo*lo, about 2^-16 of the rest, is
// dropped).  This is the starting point of the float descent state; the double
// beta0 needed by the double-precision check is computed separately.
//
// The GEMM is [K x P Wp] . [P Wp x L] with the reduction index r = (p, tau),
// tau padded to Wp = 32 ceil(W / 32) with zero atom entries.  A (the atoms)
// comes pre-split from Dsp = {hi, lo}[p][Kp][Wp] (Kp = 32 ceil(K / 32)): one
// 16-byte load per lane.  B is the Hankel matrix Y[p][t + tau]: lane (j, g)
// of a 16x16x32 tile needs Y[p][t_j + tau0 + 8 g .. + 7], a window that is
// not 16-byte aligned.  Per channel the block stages 8 copies of its signal
// window, copy sigma shifted by sigma elements (it holds Y[t_a + u + sigma] at
// u); tile starts and tau0 are multiples of 8, so lane j always reads copy
// j mod 8 at a multiple of 8: one 16-byte LDS read per operand.  A copy
// stride of 8 (mod 64) elements puts the 8 copies' reads in distinct banks.
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_rne(float x)
{
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_value(unsigned short h)
{
    return __uint_as_float((unsigned)h << 16);
}

__host__ __device__ inline int bf_pad_w(int W) { return (W + 31) / 32 * 32; }
__host__ __device__ inline int bf_pad_k(int K) { return (K + 31) / 32 * 32; }
// elements per staged copy: >= 256 + Wp, = 8 (mod 64)
__host__ __device__ inline int bf_copy_stride(int W) { return (256 + bf_pad_w(W) + 63) / 64 * 64 + 8; }

size_t corr_bf16_dsp_elems(int K, int P, int W)
{
    return 2 * (size_t)P * bf_pad_k(K) * bf_pad_w(W);
}

__global__ void __launch_bounds__(256)
k_split_d(const float* __restrict__ D, int K, int P, int W, unsigned short* __restrict__ Dsp)
{
    const int Kp = bf_pad_k(K), Wp = bf_pad_w(W);
    const size_t n = (size_t)P * Kp * Wp;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int tau = (int)(i % Wp);
        const size_t r = i / Wp;
        const int k = (int)(r % Kp);
        const int p = (int)(r / Kp);
        const float x = (k < K && tau < W) ? D[((size_t)k * P + p) * W + tau] : 0.f;
        const unsigned short h = bf16_rne(x);
        Dsp[i] = h;
        Dsp[n + i] = bf16_rne(x - bf16_value(h));
    }
}

hipError_t launch_split_d(const float* D, int K, int P, int W, unsigned short* Dsp,
                          hipStream_t s)
{
    const size_t n = corr_bf16_dsp_elems(K, P, W) / 2;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_split_d, dim3((unsigned)blocks), dim3(256), 0, s, D, K, P, W, Dsp);
    return hipGetLastError();
}

constexpr int kBfGroups = 3;   // staged signal groups (8 elements) per thread and batch
constexpr int kBfDChunks = 4;  // staged 16-byte atom chunks per thread and batch

static size_t corr_bf16_lds(int W)
{
    // 8 shifted signal copies {hi, lo} + the channel's atom slice {hi, lo}[32][Wp + 8]
    return sizeof(unsigned short) * (2 * 8 * (size_t)bf_copy_stride(W) +
                                     2 * 32 * (size_t)(bf_pad_w(W) + 8));
}

__global__ void __launch_bounds__(256)
k_corr_bf16x3(const unsigned short* __restrict__ Dsp, int K, int P, int W,
              const float* __restrict__ Y, const SigDesc* __restrict__ sig,
              const int64_t* __restrict__ tile_pref, int n_sig, float* __restrict__ g32)
{
    extern __shared__ __align__(16) unsigned short ysh[];  // [hi, lo][sigma][cs], then atoms
    const int Kp = bf_pad_k(K), Wp = bf_pad_w(W), cs = bf_copy_stride(W);
    const size_t dn = (size_t)P * Kp * Wp;  // offset of the lo half of Dsp

    const int64_t tile = blockIdx.x;
    const int si = find_sig(tile_pref, n_sig, tile);
    const SigDesc sd = sig[si];
    const int64_t t_a = (tile - tile_pref[si]) * kTile;
    const int kbase = blockIdx.y * 32;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int j = lane & 15;  // tile row (A) / column (B)
    const int g = lane >> 4;  // reduction octet

    f4_t acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            acc[a][b] = f4_t{0.f, 0.f, 0.f, 0.f};

    // Per channel the block stages the 8 shifted copies of its signal window
    // (group idx = (sigma, a) holds Y[t_a + 8 a + sigma + e], e < 8) and the
    // channel's atom slice {hi, lo}[32][Wp] (rows padded to ds = Wp + 8
    // elements: 16-byte reads of 8 consecutive rows hit distinct banks); all
    // loads are at valid (clamped) indices and unconditional, so they are in
    // flight together, and the products read LDS only.
    const int na = cs / 8;  // 8-element groups per copy
    const int ng = 8 * na;
    const int ds = Wp + 8;
    unsigned short* __restrict__ dsh = ysh + 16 * cs;  // [hi, lo][32][ds]
    const int nq = 2 * 32 * (Wp / 8);                 // 16-byte chunks of the atom slice
    const int yoff = (j & 7) * cs + 64 * wave + 8 * (j >> 3) + 8 * g;
    for (int p = 0; p < P; ++p) {
        __syncthreads();  // the previous channel's operands are consumed
        const float* __restrict__ yr = Y + sd.x_off + (int64_t)p * sd.T;
        for (int i0 = 0; i0 < ng; i0 += 256 * kBfGroups) {
            float yv[kBfGroups][8];
#pragma unroll
            for (int q = 0; q < kBfGroups; ++q) {
                const int idx = i0 + tid + 256 * q;
                const int sg = idx / na;
                const int64_t u0 = t_a + 8 * (idx - sg * na) + sg;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    yv[q][e] = yr[u0 + e < sd.T ? u0 + e : sd.T - 1];
            }
#pragma unroll
            for (int q = 0; q < kBfGroups; ++q) {
                const int idx = i0 + tid + 256 * q;
                if (idx >= ng)
                    continue;
                const int sg = idx / na;
                const int a = idx - sg * na;
                const int64_t u0 = t_a + 8 * a + sg;
                u16x8_t h, l;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float y = u0 + e < sd.T ? yv[q][e] : 0.f;
                    const unsigned short hh = bf16_rne(y);
                    h[e] = hh;
                    l[e] = bf16_rne(y - bf16_value(hh));
                }
                *reinterpret_cast<u16x8_t*>(ysh + sg * cs + 8 * a) = h;
                *reinterpret_cast<u16x8_t*>(ysh + (8 + sg) * cs + 8 * a) = l;
            }
        }
        {
            const unsigned short* __restrict__ src = Dsp + ((size_t)p * Kp + kbase) * Wp;
            for (int q0 = 0; q0 < nq; q0 += 256 * kBfDChunks) {
                u16x8_t v[kBfDChunks];
#pragma unroll
                for (int c = 0; c < kBfDChunks; ++c) {
                    int q = q0 + tid + 256 * c;
                    q = q < nq ? q : nq - 1;
                    const int hl = q / (nq / 2);
                    const int r = q - hl * (nq / 2);
                    v[c] = *reinterpret_cast<const u16x8_t*>(src + hl * dn + (size_t)r * 8);
                }
#pragma unroll
                for (int c = 0; c < kBfDChunks; ++c) {
                    const int q = q0 + tid + 256 * c;
                    if (q >= nq)
                        continue;
                    const int hl = q / (nq / 2);
                    const int r = q - hl * (nq / 2);  // row r / (Wp / 8), octet r % (Wp / 8)
                    const int row = r / (Wp / 8);
                    const int oc = r - row * (Wp / 8);
                    *reinterpret_cast<u16x8_t*>(dsh + (hl * 32 + row) * ds + 8 * oc) = v[c];
                }
            }
        }
        __syncthreads();
        // A[i][k] (atom i, reduction k) and B[k][j] (position j) sit in lane
        // i (or j) + 16 * (k / 8), element k % 8
        const unsigned short* __restrict__ yh = ysh + yoff;
        const unsigned short* __restrict__ yl = yh + 8 * cs;
        const unsigned short* __restrict__ ah = dsh + j * ds + 8 * g;
        const unsigned short* __restrict__ al = ah + 32 * ds;
        for (int t0 = 0; t0 < Wp; t0 += 32) {
            const bf16x8_t ah0 = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(ah + t0));
            const bf16x8_t al0 = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(al + t0));
            const bf16x8_t ah1 =
                __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(ah + 16 * ds + t0));
            const bf16x8_t al1 =
                __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(al + 16 * ds + t0));
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const bf16x8_t bhv =
                    __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(yh + 16 * nt + t0));
                const bf16x8_t blv =
                    __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(yl + 16 * nt + t0));
                acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, bhv, acc[0][nt], 0, 0, 0);
                acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah0, blv, acc[0][nt], 0, 0, 0);
                acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al0, bhv, acc[0][nt], 0, 0, 0);
                acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, bhv, acc[1][nt], 0, 0, 0);
                acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah1, blv, acc[1][nt], 0, 0, 0);
                acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al1, bhv, acc[1][nt], 0, 0, 0);
            }
        }
    }
    // C[i][j] of a 16x16 f32-accumulating MFMA tile sits in lane (i / 4) * 16 + j,
    // item i % 4 (measured on gfx950).
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = kbase + mi * 16 + 4 * g + v;
                const int64_t t = t_a + wave * 64 + nt * 16 + j;
                if (k < K && t < sd.L)
                    g32[sd.z_off + (int64_t)k * sd.L + t] = acc[mi][nt][v];
            }
}

hipError_t launch_corr_bf16x3(const unsigned short* Dsp, int K, int P, int W, const float* Y,
                              const SigDesc* sig, const int64_t* tile_pref, int n_sig,
                              int64_t n_tiles, float* g32, hipStream_t s)
{
    const size_t lds = corr_bf16_lds(W);
    if (lds > kLdsBytes)
        return hipErrorInvalidValue;
    if (n_tiles <= 0)
        return hipSuccess;
    (void)hipFuncSetAttribute((const void*)k_corr_bf16x3,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    dim3 grid((unsigned)n_tiles, (unsigned)(bf_pad_k(K) / 32));
    hipLaunchKernelGGL(k_corr_bf16x3, grid, dim3(256), lds, s, Dsp, K, P, W, Y, sig, tile_pref,
                       n_sig, g32);
    return hipGetLastError();
}

// lambda_max made exact: every coordinate whose float beta is within the
// float error margin of the float maximum is recomputed in double, and the
// per-signal maximum of those exact values is kept.
__global__ void __launch_bounds__(256)
k_refine_absmax(const float* __restrict__ beta32, const double* __restrict__ D,
                const float* __restrict__ X, int K, int P, int W,
                const SigDesc* __restrict__ sig, const int64_t* __restrict__ tile_pref,
                int n_sig, const double* __restrict__ thr,
                unsigned long long* __restrict__ out_bits)
{
    const int64_t tile = blockIdx.x;
    const int si = find_sig(tile_pref, n_sig, tile);
    const SigDesc sd = sig[si];
    const int64_t n = (int64_t)K * sd.L;
    const int64_t i0 = (tile - tile_pref[si]) * kAbsChunk;
    for (int64_t i = i0 + threadIdx.x; i < n && i < i0 + kAbsChunk; i += 256) {
        if (fabs((double)beta32[sd.z_off + i]) < thr[si])
            continue;
        const int k = (int)(i / sd.L);
        const int64_t t = i - (int64_t)k * sd.L;
        double acc = 0.0;
        for (int p = 0; p < P; ++p) {
            const double* dr = D + ((int64_t)k * P + p) * W;
            const float* xr = X + sd.x_off + (int64_t)p * sd.T + t;
            for (int tau = 0; tau < W; ++tau)
                acc += dr[tau] * (double)xr[tau];
        }
        atomicMax(&out_bits[si], (unsigned long long)__double_as_longlong(fabs(acc)));
    }
}

hipError_t launch_refine_absmax(const float* beta32, const double* D, const float* X, int K,
                                int P, int W, const SigDesc* sig, const int64_t* tile_pref,
                                int n_sig, int64_t n_tiles, const double* thr,
                                unsigned long long* out_bits, hipStream_t s)
{
    hipLaunchKernelGGL(k_refine_absmax, dim3((unsigned)n_tiles), dim3(256), 0, s, beta32, D, X,
                       K, P, W, sig, tile_pref, n_sig, thr, out_bits);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dictionary finish: float copy of S, norms |D_k|^2 = S_{k,k}[0] and inverses.
// ---------------------------------------------------------------------------
__global__ void k_dict_finish(const double* __restrict__ S64, int K, int W,
                              float* __restrict__ S32, double* __restrict__ n2_64,
                              double* __restrict__ inv64, float* __restrict__ n2_32,
                              float* __restrict__ inv32)
{
    const int nd = 2 * W - 1;
    const size_t n = (size_t)K * K * nd;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        S32[i] = (float)S64[i];
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)K) {
        const int k = threadIdx.x;
        const double v = S64[((size_t)k * K + k) * nd + (W - 1)];
        n2_64[k] = v;
        inv64[k] = 1.0 / v;
        n2_32[k] = (float)v;
        inv32[k] = (float)(1.0 / v);
    }
}

hipError_t launch_dict_finish(const double* S64, int K, int W, float* S32,
                              double* n2_64, double* inv_n2_64, float* n2_32,
                              float* inv_n2_32, hipStream_t s)
{
    hipLaunchKernelGGL(k_dict_finish, dim3(64), dim3(256), 0, s, S64, K, W, S32,
                       n2_64, inv_n2_64, n2_32, inv_n2_32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// lambda_max = max |beta| per signal (bit pattern of a non-negative double,
// whose unsigned order is the numeric order).
// ---------------------------------------------------------------------------


template <typename T>
__global__ void __launch_bounds__(256)
k_absmax(const T* __restrict__ beta, int K, const SigDesc* __restrict__ sig,
         const int64_t* __restrict__ tile_pref, int n_sig,
         unsigned long long* __restrict__ out_bits)
{
    __shared__ double red[4];
    const int64_t tile = blockIdx.x;
    const int si = find_sig(tile_pref, n_sig, tile);
    const SigDesc sd = sig[si];
    const int64_t n = (int64_t)K * sd.L;
    const int64_t i0 = (tile - tile_pref[si]) * kAbsChunk;
    double m = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < n && i < i0 + kAbsChunk; i += 256)
        m = fmax(m, fabs((double)beta[sd.z_off + i]));
    for (int o = 32; o > 0; o >>= 1)
        m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        atomicMax(&out_bits[si], (unsigned long long)__double_as_longlong(m));
    }
}

hipError_t launch_absmax(const double* beta, int K, const SigDesc* sig,
                         const int64_t* tile_pref, int n_sig, int64_t n_tiles,
                         unsigned long long* out_bits, hipStream_t s)
{
    hipLaunchKernelGGL(k_absmax<double>, dim3((unsigned)n_tiles), dim3(256), 0, s,
                       beta, K, sig, tile_pref, n_sig, out_bits);
    return hipGetLastError();
}

// Gap Safe sphere rule at the current Z (safe screening): coordinate (k, t)
// is zero in every solution when |g_k[t]| / s + r |D_k| < 1, with g = D^T R,
// s = max(lambda, max |g|) and r = sqrt(2 gap) / lambda per signal
// (rule[2 si] = 1 / s, rule[2 si + 1] = r).  A float g is enlarged by 2^-22
// of itself first, so rounding never screens a coordinate the double value
// would keep.  count[si] gets the screened coordinates.
template <typename T>
__global__ void __launch_bounds__(256)
k_screen_count(const T* __restrict__ g, const double* __restrict__ n2, int K,
               const SigDesc* __restrict__ sig, const int64_t* __restrict__ tile_pref,
               int n_sig, const double* __restrict__ rule,
               unsigned long long* __restrict__ count)
{
    __shared__ unsigned long long red[4];
    const int64_t tile = blockIdx.x;
    const int si = find_sig(tile_pref, n_sig, tile);
    const SigDesc sd = sig[si];
    const int64_t n = (int64_t)K * sd.L;
    const int64_t i0 = (tile - tile_pref[si]) * kAbsChunk;
    const double inv_s = rule[2 * si], r = rule[2 * si + 1];
    const double slack = sizeof(T) == 4 ? 2.384185791015625e-7 : 0.0;  // 2^-22
    unsigned long long c = 0;
    for (int64_t i = i0 + threadIdx.x; i < n && i < i0 + kAbsChunk; i += 256) {
        const int k = (int)(i / sd.L);
        const double a = fabs((double)g[sd.z_off + i]);
        c += (a + slack * a) * inv_s + r * sqrt(n2[k]) < 1.0 ? 1ull : 0ull;
    }
    for (int o = 32; o > 0; o >>= 1)
        c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicAdd(&count[si], red[0] + red[1] + red[2] + red[3]);
}

hipError_t launch_screen_count(const void* g, bool fp64, const double* n2, int K,
                               const SigDesc* sig, const int64_t* tile_pref, int n_sig,
                               int64_t n_tiles, const double* rule, unsigned long long* count,
                               hipStream_t s)
{
    if (fp64)
        hipLaunchKernelGGL(k_screen_count<double>, dim3((unsigned)n_tiles), dim3(256), 0, s,
                           (const double*)g, n2, K, sig, tile_pref, n_sig, rule, count);
    else
        hipLaunchKernelGGL(k_screen_count<float>, dim3((unsigned)n_tiles), dim3(256), 0, s,
                           (const float*)g, n2, K, sig, tile_pref, n_sig, rule, count);
    return hipGetLastError();
}

hipError_t launch_absmax_f32(const float* beta, int K, const SigDesc* sig,
                             const int64_t* tile_pref, int n_sig, int64_t n_tiles,
                             unsigned long long* out_bits, hipStream_t s)
{
    hipLaunchKernelGGL(k_absmax<float>, dim3((unsigned)n_tiles), dim3(256), 0, s,
                       beta, K, sig, tile_pref, n_sig, out_bits);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LGCD phase kernel: one workgroup runs the locally greedy descent of one
// segment C_m (Algorithm 3 restricted to that segment) until its largest
// |Delta Z| is below eps_stop or `cap` updates were applied.
//
// LDS holds g for the segment extended by W - 1 positions on each side (the
// "interference zone" of Sec. 2.2) and a copy of Z for the segment, both
// position-major with the atoms of one position contiguous (padded to a
// multiple of 16 bytes).  The correlation table is read in the matching
// layout St[k0][d][k], so the eq. (3) update of one position is a few 16-byte
// loads, one multiply-add per atom and 16-byte stores.  Thread tid owns the
// extended positions q = tid + i * 512; every LDS entry is read and written
// only by its owner, so the window update needs no synchronisation.  The
// argmax is a block reduction of the per-position best (|Delta Z|, t * K + k)
// keys; ties go to the smallest t, then k.  Each update costs one barrier.
//
// Segments of one parity run in the same launch.  A run writes g back over
// the part of the extended window it touched, i.e. into the idle neighbours'
// positions: this is the even/odd form of the boundary messages of
// Algorithm 2.  Segments are at least W - 1 long and same-colour segments are
// at least 2W - 2 apart, so two runs of one launch never touch the same entry.
// ---------------------------------------------------------------------------

template <typename G>
struct Vec;
template <>
struct Vec<float> {
    typedef float T __attribute__((ext_vector_type(4)));
    static constexpr int N = 4;
};
template <>
struct Vec<double> {
    typedef double T __attribute__((ext_vector_type(2)));
    static constexpr int N = 2;
};

// Argmax keys.  float state: one 64-bit word, |Delta Z| bits above the
// complemented index, so a plain unsigned max picks the largest value and,
// among equal values, the smallest index.  double state: value bits and index
// in two words.
struct Key64 {
    unsigned long long v;  // bit pattern of |Delta Z| (non-negative double)
    unsigned int i;        // j * K + k inside the segment
};

template <typename G>
struct KeyOps;

// One DPP step of a wave-wide maximum of a 64-bit unsigned key: the lanes in
// rows enabled by RM read the lane selected by CTRL; others keep their value.
template <int CTRL, int RM>
__device__ __forceinline__ unsigned long long dpp_max_step(unsigned long long a)
{
    const unsigned lo = (unsigned)a, hi = (unsigned)(a >> 32);
    const unsigned olo = (unsigned)__builtin_amdgcn_update_dpp((int)lo, (int)lo, CTRL, RM, 0xf, false);
    const unsigned ohi = (unsigned)__builtin_amdgcn_update_dpp((int)hi, (int)hi, CTRL, RM, 0xf, false);
    const unsigned long long o = ((unsigned long long)ohi << 32) | olo;
    return o > a ? o : a;
}

// Wave-wide maximum with DPP row operations: quad swaps, half-row and row
// mirrors, then the row broadcasts of lanes 15 and 31; lane 63 ends with the
// maximum of all 64 lanes, which is broadcast through a scalar register.
__device__ __forceinline__ unsigned long long dpp_wave_max_u64(unsigned long long a)
{
    a = dpp_max_step<0xB1, 0xf>(a);   // quad_perm [1,0,3,2]
    a = dpp_max_step<0x4E, 0xf>(a);   // quad_perm [2,3,0,1]
    a = dpp_max_step<0x141, 0xf>(a);  // row_half_mirror
    a = dpp_max_step<0x140, 0xf>(a);  // row_mirror
    a = dpp_max_step<0x142, 0xa>(a);  // row_bcast:15 into rows 1 and 3
    a = dpp_max_step<0x143, 0xc>(a);  // row_bcast:31 into rows 2 and 3
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)a, 63);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(a >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

template <>
struct KeyOps<float> {
    typedef unsigned long long T;
    static __device__ __forceinline__ T null() { return 0ull; }
    static __device__ __forceinline__ T make(float ad, unsigned idx)
    {
        return ((unsigned long long)__float_as_uint(ad) << 32) |
               (unsigned long long)(0xffffffffu - idx);
    }
    static __device__ __forceinline__ bool better(T a, T b) { return a > b; }
    static __device__ __forceinline__ double value(T a)
    {
        return (double)__uint_as_float((unsigned)(a >> 32));
    }
    static __device__ __forceinline__ unsigned index(T a)
    {
        return 0xffffffffu - (unsigned)(a & 0xffffffffull);
    }
    static __device__ __forceinline__ T wave_max(T a) { return dpp_wave_max_u64(a); }
    static __device__ __forceinline__ bool same(T a, T b) { return a == b; }
    static __device__ __forceinline__ T select(bool c, T a, T b) { return c ? a : b; }
};

template <>
struct KeyOps<double> {
    typedef Key64 T;
    static __device__ __forceinline__ T null() { return Key64{0ull, 0xffffffffu}; }
    static __device__ __forceinline__ T make(double ad, unsigned idx)
    {
        return Key64{(unsigned long long)__double_as_longlong(ad), idx};
    }
    static __device__ __forceinline__ bool better(const T& a, const T& b)
    {
        return a.v > b.v || (a.v == b.v && a.i < b.i);
    }
    static __device__ __forceinline__ double value(const T& a)
    {
        return __longlong_as_double((long long)a.v);
    }
    static __device__ __forceinline__ unsigned index(const T& a) { return a.i; }
    static __device__ __forceinline__ T wave_max(T a)
    {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            T b;
            b.v = __shfl_xor(a.v, o);
            b.i = __shfl_xor(a.i, o);
            const bool t = better(b, a);
            a.v = t ? b.v : a.v;
            a.i = t ? b.i : a.i;
        }
        return a;
    }
    static __device__ __forceinline__ bool same(const T& a, const T& b)
    {
        return a.v == b.v && a.i == b.i;
    }
    static __device__ __forceinline__ T select(bool c, const T& a, const T& b)
    {
        return Key64{c ? a.v : b.v, c ? a.i : b.i};
    }
};

template <typename G>
struct Slot {
    typename KeyOps<G>::T key;
    G d;
};

// Delta Z = Z' - Z in terms of g (eq. (pb_coord) with beta = g + |D|^2 z):
// -z where the soft threshold sends the coordinate to 0 (*zero), else
// (g - lambda sign(beta)) / |D|^2, formed as g * inv - copysign(lambda * inv,
// beta) with lam_inv = lambda * inv (no cancellation against z).
template <typename G>
__device__ __forceinline__ G coord_delta(G g, G z, G n2, G inv_n2, G lam_inv, G lam,
                                         bool* zero)
{
    const G bb = fma(n2, z, g);
    const bool zr = fabs(bb) <= lam;
    *zero = zr;
    return zr ? -z : fma(g, inv_n2, -copysign(lam_inv, bb));
}

// Block argmax over every thread's NQ position keys; returns the winner's key
// and Delta Z in all threads.  One barrier; slots are double-buffered by the
// caller.
template <typename G, int NQ, int NT = kPhaseThreads>
__device__ __forceinline__ void block_argmax(const typename KeyOps<G>::T (&best)[NQ],
                                             const G (&dl)[NQ], Slot<G>* __restrict__ slot,
                                             typename KeyOps<G>::T& out, G& dout)
{
    typedef KeyOps<G> KO;
    constexpr int NW = NT / 64;
    typename KO::T m = best[0];
    G d = dl[0];
    static_for<NQ>([&](auto ic) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        if (i > 0) {
            const bool b = KO::better(best[i], m);
            m = KO::select(b, best[i], m);
            d = b ? dl[i] : d;
        }
    });
    const typename KO::T w = KO::wave_max(m);
    if (KO::same(m, w)) {
        slot[threadIdx.x >> 6].key = w;
        slot[threadIdx.x >> 6].d = d;
    }
    __syncthreads();
    typename KO::T bb = slot[0].key;
    G bd = slot[0].d;
#pragma unroll
    for (int wv = 1; wv < NW; ++wv) {
        const typename KO::T o = slot[wv].key;
        const bool b = KO::better(o, bb);
        bb = KO::select(b, o, bb);
        bd = b ? slot[wv].d : bd;
    }
    out = bb;
    dout = bd;
}

// One extended position: optional eq. (3) update g -= S delta (s_row != null)
// and, for an own position (z_row != null), the best candidate over the atoms.
// Padded atoms have g = z = S = 0 and |D|^2 = 1, so their candidate is 0.
template <typename G, int KQ>
__device__ __forceinline__ void load_s_row(const G* __restrict__ s_row,
                                           typename Vec<G>::T (&sv)[KQ])
{
#pragma unroll
    for (int i = 0; i < KQ; ++i)
        sv[i] = reinterpret_cast<const typename Vec<G>::T*>(s_row)[i];
}

// upd: apply g -= S delta with the S row given in sv (loaded by the caller,
// early when it can be).
template <typename G, int KQ>
__device__ __forceinline__ void visit(G* __restrict__ g_row, const G* __restrict__ z_row,
                                      bool upd, const typename Vec<G>::T (&sv)[KQ], G delta,
                                      const G (&n2r)[KQ * Vec<G>::N],
                                      const G (&invr)[KQ * Vec<G>::N],
                                      const G (&linvr)[KQ * Vec<G>::N],
                                      const G* __restrict__ n2l, const G* __restrict__ invl,
                                      const G* __restrict__ linvl, G lam, unsigned idx_base,
                                      typename KeyOps<G>::T& key, G& dbest)
{
    typedef typename Vec<G>::T V;
    constexpr int N = Vec<G>::N;
    V gv[KQ], zv[KQ];
#pragma unroll
    for (int i = 0; i < KQ; ++i)
        gv[i] = reinterpret_cast<const V*>(g_row)[i];
    if (z_row) {
#pragma unroll
        for (int i = 0; i < KQ; ++i)
            zv[i] = reinterpret_cast<const V*>(z_row)[i];
    }
    if (upd) {
#pragma unroll
        for (int i = 0; i < KQ; ++i) {
            gv[i] -= sv[i] * delta;
            reinterpret_cast<V*>(g_row)[i] = gv[i];
        }
    }
    if (z_row) {
        G bestv = (G)-1;
        int bk = 0;
#pragma unroll
        for (int i = 0; i < KQ; ++i) {
            // per-atom constants: vector registers in float up to 28 atoms;
            // otherwise (too many registers) 16-byte LDS broadcast reads
            V nv, iv, lv;
            if (sizeof(G) == sizeof(float) && KQ <= 7) {
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    nv[c] = n2r[i * N + c];
                    iv[c] = invr[i * N + c];
                    lv[c] = linvr[i * N + c];
                }
            } else {
                nv = reinterpret_cast<const V*>(n2l)[i];
                iv = reinterpret_cast<const V*>(invl)[i];
                lv = reinterpret_cast<const V*>(linvl)[i];
            }
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const int k = i * N + c;
                bool zr;
                const G d = coord_delta<G>(gv[i][c], zv[i][c], nv[c], iv[c], lv[c], lam, &zr);
                const G ad = fabs(d);
                const bool b = ad > bestv;
                bestv = b ? ad : bestv;
                bk = b ? k : bk;
            }
        }
        key = KeyOps<G>::make(bestv, idx_base + (unsigned)bk);
        // the signed change of the winning atom, recomputed from the stored state
        bool zr;
        dbest = coord_delta<G>(g_row[bk], z_row[bk], n2l[bk], invl[bk], linvl[bk], lam, &zr);
    }
}

// An update whose window reaches a neighbour (the halo), kept until the end
// of the run: (atom, signal position, applied change).
template <typename G>
struct HaloRec {
    int k0;
    int t0;
    G delta;
};
constexpr int kHaloRecs = 64;  // records held on chip before they are applied

// Byte offset of the argmax slots after the g and Z arrays, 16-byte aligned.
__host__ __device__ constexpr size_t slot_offset(size_t elem, int KP, int lx, int lm)
{
    return ((elem * (size_t)KP * ((size_t)lx + (size_t)lm)) + 15) & ~(size_t)15;
}

template <typename G, int KQ, int NQ, int NT, bool DI>
__global__ void __launch_bounds__(NT)
k_lgcd_phase(PhaseArgs a)
{
    typedef KeyOps<G> KO;
    typedef typename KO::T KeyT;
    typedef typename Vec<G>::T V;
    constexpr int NW = NT / 64;
    constexpr int KP = KQ * Vec<G>::N;
    const int K = a.K;
    const int W = a.W;
    const int nd = 2 * W - 1;
    const int tid = threadIdx.x;

    const int sid = a.list[blockIdx.x];
    // DI (Algorithm 2 in lockstep): flags and boxes of this phase's parity
    const int par = a.phase & 1;
    uint32_t* dirty = DI ? a.dirty + (size_t)par * a.n_seg : a.dirty;
    uint32_t* msg_n_out = DI ? a.msg_n + ((size_t)par * a.n_seg + sid) * 2 : nullptr;
    if (DI && tid == 0) {
        msg_n_out[0] = 0u;  // rewritten below when the segment runs
        msg_n_out[1] = 0u;
    }
    if (dirty[sid] == 0)
        return;

    extern __shared__ __align__(16) unsigned char smem[];
    const SegDesc sd = a.segs[sid];
    const int64_t L = sd.L;
    const int b = sd.b;
    const int Lm = sd.e - sd.b;
    // The halo: the neighbours' positions within W - 1 of the segment.  The
    // block keeps only its own positions (index j = t - b) on chip; an
    // update's change of the halo is recorded and applied to the state in HBM
    // at the end of the run (the neighbours are idle in this phase).  DI: no
    // halo, the neighbours get messages.
    const int ext_lo = DI ? b : (b - (W - 1) > 0 ? b - (W - 1) : 0);
    const int ext_hi = DI ? sd.e : (sd.e + (W - 1) < sd.L ? sd.e + (W - 1) : sd.L);
    const int lm = a.lm_max;

    G* g_l = reinterpret_cast<G*>(smem);          // [lm][KP]
    G* z_l = g_l + (size_t)lm * KP;               // [lm][KP]
    Slot<G>* slots = reinterpret_cast<Slot<G>*>(smem + slot_offset(sizeof(G), KP, lm, lm));
    G* n2l = reinterpret_cast<G*>(slots + 2 * NW);  // [KP]
    G* invl = n2l + KP;                             // [KP]
    G* linvl = invl + KP;                           // [KP] lambda / |D_k|^2
    HaloRec<G>* recs = reinterpret_cast<HaloRec<G>*>(
        reinterpret_cast<unsigned char*>(linvl + KP) +
        ((16 - (reinterpret_cast<size_t>(linvl + KP) & 15)) & 15));  // [kHaloRecs]

    G* __restrict__ gs = reinterpret_cast<G*>(a.g) + sd.z_off;
    double* __restrict__ Zs = a.Z + sd.z_off;
    const G* __restrict__ St = reinterpret_cast<const G*>(a.S);  // [K][nd][KP]
    const G lam = (G)a.sigs[sd.sig].lam;
    const double eps_stop = a.sigs[sd.sig].eps_stop;

    // |D_k|^2, its inverse and lambda times it: in LDS for the data-dependent
    // updated atom, and copied to vector registers (per-thread copies: the
    // per-position passes use all of them) after the barrier below.  Padded
    // atoms get 1.
    for (int k = tid; k < KP; k += NT) {
        const G iv = k < K ? reinterpret_cast<const G*>(a.inv_n2)[k] : (G)1;
        n2l[k] = k < K ? reinterpret_cast<const G*>(a.n2)[k] : (G)1;
        invl[k] = iv;
        linvl[k] = lam * iv;
    }
    // own state in: [k][t] in HBM -> [j][k] in LDS, padding zeroed (loads at
    // clamped, valid atoms: unconditional, so that several are in flight)
#pragma unroll 4
    for (int i = tid; i < KP * Lm; i += NT) {
        const int k = i / Lm;
        const int j = i - k * Lm;
        const int kc = k < K ? k : K - 1;
        const G gv = gs[(int64_t)kc * L + b + j];
        const G zv = (G)Zs[(int64_t)kc * L + b + j];
        g_l[j * KP + k] = k < K ? gv : (G)0;
        z_l[j * KP + k] = k < K ? zv : (G)0;
    }
    __syncthreads();
    G n2r[KP], invr[KP], linvr[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        n2r[k] = n2l[k];
        invr[k] = invl[k];
        linvr[k] = linvl[k];
    }
    int tlo = INT_MAX, thi = -1;  // own positions whose g changed (written back)
    if (DI) {
        // messages of the previous phase: the left neighbour's rightwards box,
        // then the right neighbour's leftwards box, each in the order sent;
        // every position is changed by its owner thread only
        const int prev = par ^ 1;
        for (int side = 0; side < 2; ++side) {
            const int nb = side == 0 ? sd.left : sd.right;
            if (nb < 0)
                continue;
            const size_t box = ((size_t)prev * a.n_seg + nb) * 2 + (side == 0 ? 1 : 0);
            const uint32_t cnt = a.msg_n[box];
            const DicodMsg* mb = a.msg + box * a.msg_cap;
            for (uint32_t i = 0; i < cnt; ++i) {
                const DicodMsg mg = mb[i];
                const int j0m = mg.t0 - b;
                const G dm = (G)mg.delta;
                const int mlo = j0m - (W - 1) > 0 ? j0m - (W - 1) : 0;
                const int mhi = j0m + (W - 1) < Lm - 1 ? j0m + (W - 1) : Lm - 1;
                tlo = mlo < tlo ? mlo : tlo;
                thi = mhi > thi ? mhi : thi;
                const G* __restrict__ Sk = St + (size_t)mg.k0 * nd * KP;
                static_for<NQ>([&](auto ic) __attribute__((always_inline)) {
                    constexpr int i2 = decltype(ic)::value;
                    const int j = tid + i2 * NT;
                    const int dj = j - j0m + (W - 1);
                    if (j >= Lm || dj < 0 || dj >= nd)
                        return;
                    KeyT kd = KO::null();
                    G dd = (G)0;
                    V sv[KQ];
                    load_s_row<G, KQ>(Sk + (size_t)dj * KP, sv);
                    visit<G, KQ>(g_l + j * KP, nullptr, true, sv, dm, n2r, invr, linvr, n2l,
                                 invl, linvl, lam, 0u, kd, dd);
                });
            }
        }
    }

    // Halo records recs[0..cnt) applied to the state in HBM, each halo
    // position by one thread, records in update order (the same operations
    // in the same order as applying them at each update); atoms in groups of
    // four vectors to bound the registers.
    auto flush_halo = [&](int cnt) __attribute__((always_inline)) {
        constexpr int GV = KQ < 4 ? KQ : 4;
        const int n_hl = b - ext_lo;
        const int n_h = n_hl + (ext_hi - sd.e);
        for (int h = tid; h < n_h; h += NT) {
            const int t = h < n_hl ? ext_lo + h : sd.e + (h - n_hl);
#pragma unroll
            for (int c0 = 0; c0 < KQ; c0 += GV) {
                bool touched = false;
                V gv[GV];
                for (int r = 0; r < cnt; ++r) {
                    const HaloRec<G> rc = recs[r];
                    const int dj = t - rc.t0 + (W - 1);
                    if (dj < 0 || dj >= nd)
                        continue;
                    if (!touched) {
#pragma unroll
                        for (int c = 0; c < GV; ++c)
#pragma unroll
                            for (int e = 0; e < Vec<G>::N; ++e) {
                                const int k = (c0 + c) * Vec<G>::N + e;
                                const G v = gs[(int64_t)(k < K ? k : K - 1) * L + t];
                                gv[c][e] = (c0 + c < KQ && k < K) ? v : (G)0;
                            }
                        touched = true;
                    }
                    const V* srow = reinterpret_cast<const V*>(
                        St + ((size_t)rc.k0 * nd + dj) * KP);
#pragma unroll
                    for (int c = 0; c < GV; ++c)
                        if (c0 + c < KQ)
                            gv[c] -= srow[c0 + c] * rc.delta;
                }
                if (touched) {
#pragma unroll
                    for (int c = 0; c < GV; ++c)
#pragma unroll
                        for (int e = 0; e < Vec<G>::N; ++e) {
                            const int k = (c0 + c) * Vec<G>::N + e;
                            if (c0 + c < KQ && k < K)
                                gs[(int64_t)k * L + t] = gv[c][e];
                        }
                }
            }
        }
    };

    KeyT best[NQ];
    G dl[NQ];
    static_for<NQ>([&](auto ic) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        best[i] = KO::null();
        dl[i] = (G)0;
        const int j = tid + i * NT;
        if (j < Lm) {
            V sv[KQ];  // unused: no update in this pass
            visit<G, KQ>(g_l + j * KP, z_l + j * KP, false, sv, (G)0, n2r, invr, linvr, n2l,
                         invl, linvl, lam, (unsigned)(j * KP), best[i], dl[i]);
        }
    });

    int it = 0;
    KeyT kb;
    G db;
    block_argmax<G, NQ, NT>(best, dl, slots + (it & 1) * NW, kb, db);
    ++it;

    int n = 0, nrec = 0;
    bool conv = false;
    bool touch_l = false, touch_r = false;
    unsigned n_msg_l = 0, n_msg_r = 0;
    for (;;) {
        if (KO::value(kb) < eps_stop) {
            conv = true;
            break;
        }
        if (n == a.cap)
            break;
        const unsigned kidx = KO::index(kb);
        const int j0 = (int)(kidx / (unsigned)KP);  // keys index j * KP + k
        const int k0 = (int)kidx - j0 * KP;
        const G delta = db;
        const int wlo = j0 - (W - 1) > 0 ? j0 - (W - 1) : 0;
        const int whi = j0 + (W - 1) < Lm - 1 ? j0 + (W - 1) : Lm - 1;
        const G* __restrict__ Sk = St + (size_t)k0 * nd * KP;

        if (tid == (j0 % NT)) {
            // Owner of the updated position: new Z value (exactly 0 when the
            // soft threshold is active), in LDS and in the double-precision Z.
            const G zo = z_l[j0 * KP + k0];
            bool zr;
            (void)coord_delta<G>(g_l[j0 * KP + k0], zo, n2l[k0], invl[k0], linvl[k0], lam, &zr);
            const G zn = zr ? (G)0 : zo + delta;
            z_l[j0 * KP + k0] = zn;
            double* zp = Zs + (int64_t)k0 * L + b + j0;
            if (sizeof(G) == sizeof(double)) {
                *zp = (double)zn;
            } else {
                if (zr)
                    *zp = 0.0;
                else
                    unsafeAtomicAdd(zp, (double)delta);  // single owner: deterministic
            }
            if (a.trace) {
                const unsigned long long r = atomicAdd(&a.counters->trace_n, 1ull);
                if ((long long)r < a.trace_cap) {
                    dicod_trace_rec rec;
                    rec.phase = a.phase;
                    rec.seg = sid;
                    rec.k0 = k0;
                    rec.n_local = n;
                    rec.t0 = (int64_t)b + j0;
                    rec.delta = zr ? -(double)zo : (double)delta;
                    a.trace[r] = rec;
                }
            }
        }

        tlo = wlo < tlo ? wlo : tlo;
        thi = whi > thi ? whi : thi;
        const bool to_l = j0 - (W - 1) < 0 && sd.left >= 0;
        const bool to_r = j0 + (W - 1) >= Lm && sd.right >= 0;
        if (tid == (j0 % NT) && (to_l || to_r)) {
            if (DI) {
                // the update as sent: the delta this segment applied to g
                DicodMsg mg;
                mg.k0 = k0;
                mg.t0 = b + j0;
                mg.delta = (double)delta;
                if (to_l)
                    a.msg[(((size_t)par * a.n_seg + sid) * 2 + 0) * a.msg_cap + n_msg_l] = mg;
                if (to_r)
                    a.msg[(((size_t)par * a.n_seg + sid) * 2 + 1) * a.msg_cap + n_msg_r] = mg;
            } else {
                HaloRec<G> rc;
                rc.k0 = k0;
                rc.t0 = b + j0;
                rc.delta = delta;
                recs[nrec] = rc;
            }
        }
        n_msg_l += to_l ? 1 : 0;
        n_msg_r += to_r ? 1 : 0;
        nrec += (!DI && (to_l || to_r)) ? 1 : 0;
        touch_l |= to_l;
        touch_r |= to_r;

        static_for<NQ>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            const int j = tid + i * NT;
            if (j < wlo || j > whi)
                return;
            V sv[KQ];
            load_s_row<G, KQ>(Sk + (size_t)(j - j0 + (W - 1)) * KP, sv);
            visit<G, KQ>(g_l + j * KP, z_l + j * KP, true, sv, delta, n2r, invr, linvr, n2l,
                         invl, linvl, lam, (unsigned)(j * KP), best[i], dl[i]);
        });
        ++n;
        block_argmax<G, NQ, NT>(best, dl, slots + (it & 1) * NW, kb, db);
        ++it;
        if (!DI && nrec == kHaloRecs) {
            // full record list (the records are visible after the barrier in
            // block_argmax): apply it, and let every thread finish reading it
            // before it is reused
            flush_halo(nrec);
            nrec = 0;
            __syncthreads();
        }
    }
    if (!DI && nrec > 0)
        flush_halo(nrec);

    if (thi >= tlo) {
        // own g of every position changed by an update or a message
        const int wdt = thi - tlo + 1;
        for (int i = tid; i < K * wdt; i += NT) {
            const int k = i / wdt;
            const int j = tlo + (i - k * wdt);
            gs[(int64_t)k * L + b + j] = g_l[j * KP + k];
        }
    }
    if (n > 0) {
        if (tid == 0) {
            atomicAdd(&a.phase_upd[(size_t)sd.sig * a.phase_stride + a.phase], (unsigned long long)n);
            atomicAdd(&a.sig_upd[sd.sig], (unsigned long long)n);
            atomicMax(&a.sig_last_upd[sd.sig], a.phase);
            atomicAdd(&a.counters->seg_runs, 1ull);
            if (a.changed)
                a.changed[sid] = 1u;
        }
    }
    if (tid == 0) {
        if (DI) {
            // this parity's flag is consumed; the next phase's flags (the other
            // parity) are only ever set here, so a neighbour's mark survives
            uint32_t* next = a.dirty + (size_t)(par ^ 1) * a.n_seg;
            dirty[sid] = 0u;
            if (!conv)
                next[sid] = 1u;
            if (touch_l)
                next[sd.left] = 1u;
            if (touch_r)
                next[sd.right] = 1u;
            msg_n_out[0] = n_msg_l;
            msg_n_out[1] = n_msg_r;
        } else {
            a.dirty[sid] = conv ? 0u : 1u;
            if (touch_l)
                a.dirty[sd.left] = 1u;
            if (touch_r)
                a.dirty[sd.right] = 1u;
        }
    }
}

// Atoms per position in the kernel instantiations: K is padded to one of
// these multiples of the 16-byte vector width.
static int pick_kq(int K, bool fp64)
{
    const int n = fp64 ? 2 : 4;
    const int need = (K + n - 1) / n;
    static const int f32[] = {1, 2, 4, 7, 8, 16};
    static const int f64[] = {1, 2, 3, 4, 8, 13, 16, 32};
    const int* t = fp64 ? f64 : f32;
    const int m = fp64 ? 8 : 6;
    for (int i = 0; i < m; ++i)
        if (t[i] >= need)
            return t[i];
    return -1;
}

int lgcd_k_padded(int K, bool fp64)
{
    const int kq = pick_kq(K, fp64);
    return kq < 0 ? -1 : kq * (fp64 ? 2 : 4);
}

size_t lgcd_lds_bytes(int K, int lm_max, int lext_max, bool fp64)
{
    (void)lext_max;  // the halo stays in HBM
    const int KP = lgcd_k_padded(K, fp64);
    if (KP < 0)
        return (size_t)-1;
    const size_t e = fp64 ? sizeof(double) : sizeof(float);
    const size_t slots = 2 * (kPhaseThreadsMax / 64) *
                         (fp64 ? sizeof(Slot<double>) : sizeof(Slot<float>));
    const size_t recs = kHaloRecs * (fp64 ? sizeof(HaloRec<double>) : sizeof(HaloRec<float>));
    return slot_offset(e, KP, lm_max, lm_max) + slots + 3 * e * (size_t)KP + 16 + recs;
}

template <typename G, int KQ, int NQ, int NT>
static hipError_t launch_phase_inst(const PhaseArgs& a, size_t lds, hipStream_t s)
{
    const void* fn = a.dicod ? (const void*)k_lgcd_phase<G, KQ, NQ, NT, true>
                             : (const void*)k_lgcd_phase<G, KQ, NQ, NT, false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    if (a.dicod)
        hipLaunchKernelGGL((k_lgcd_phase<G, KQ, NQ, NT, true>), dim3((unsigned)a.n_list),
                           dim3(NT), lds, s, a);
    else
        hipLaunchKernelGGL((k_lgcd_phase<G, KQ, NQ, NT, false>), dim3((unsigned)a.n_list),
                           dim3(NT), lds, s, a);
    return hipGetLastError();
}

// 1024-thread workgroups (one extended position per thread, four waves per
// SIMD) for float state with up to 32 atoms; 512 threads otherwise.
template <typename G, int KQ>
static hipError_t launch_phase_kq(const PhaseArgs& a, size_t lds, hipStream_t s)
{
    // 512 threads measured faster than 256 (one position per thread) and
    // than 1024 on gfx950
    constexpr bool wide = false;
    if (wide && a.lm_max <= kPhaseThreadsMax)
        return launch_phase_inst<G, KQ, 1, (wide ? kPhaseThreadsMax : kPhaseThreads)>(a, lds, s);
    switch ((a.lm_max + kPhaseThreads - 1) / kPhaseThreads) {
    case 1: return launch_phase_inst<G, KQ, 1, kPhaseThreads>(a, lds, s);
    case 2: return launch_phase_inst<G, KQ, 2, kPhaseThreads>(a, lds, s);
    case 3: return launch_phase_inst<G, KQ, 3, kPhaseThreads>(a, lds, s);
    case 4: return launch_phase_inst<G, KQ, 4, kPhaseThreads>(a, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lgcd_phase(const PhaseArgs& a, bool fp64, size_t* lds_bytes,
                             hipStream_t s)
{
    if (a.n_list <= 0)
        return hipSuccess;
    const int nq = (a.lm_max + kPhaseThreads - 1) / kPhaseThreads;
    if (nq < 1 || nq > 4)
        return hipErrorInvalidValue;
    const size_t lds = lgcd_lds_bytes(a.K, a.lm_max, a.lext_max, fp64);
    if (lds_bytes)
        *lds_bytes = lds;
    if (lds > kLdsBytes)
        return hipErrorInvalidValue;
    const int kq = pick_kq(a.K, fp64);
    if (fp64) {
        switch (kq) {
        case 1: return launch_phase_kq<double, 1>(a, lds, s);
        case 2: return launch_phase_kq<double, 2>(a, lds, s);
        case 3: return launch_phase_kq<double, 3>(a, lds, s);
        case 4: return launch_phase_kq<double, 4>(a, lds, s);
        case 8: return launch_phase_kq<double, 8>(a, lds, s);
        case 13: return launch_phase_kq<double, 13>(a, lds, s);
        case 16: return launch_phase_kq<double, 16>(a, lds, s);
        case 32: return launch_phase_kq<double, 32>(a, lds, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (kq) {
    case 1: return launch_phase_kq<float, 1>(a, lds, s);
    case 2: return launch_phase_kq<float, 2>(a, lds, s);
    case 4: return launch_phase_kq<float, 4>(a, lds, s);
    case 7: return launch_phase_kq<float, 7>(a, lds, s);
    case 8: return launch_phase_kq<float, 8>(a, lds, s);
    case 16: return launch_phase_kq<float, 16>(a, lds, s);
    default: return hipErrorInvalidValue;
    }
}

// Correlation table in the phase kernel's layout: St[l][d][k] = S_{k,l}[d-W+1]
// for k < K, zero for the padded atoms k in [K, KP).
template <typename G>
__global__ void k_s_transpose(const double* __restrict__ S64, int K, int W, int KP,
                              G* __restrict__ St)
{
    const int nd = 2 * W - 1;
    const size_t n = (size_t)K * nd * KP;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % KP);
        const size_t r = i / KP;
        const int d = (int)(r % nd);
        const int l = (int)(r / nd);
        St[i] = k < K ? (G)S64[((size_t)l * K + k) * nd + d] : (G)0;
    }
}

hipError_t launch_s_transpose(const double* S64, int K, int W, bool fp64, void* St,
                              hipStream_t s)
{
    const int KP = lgcd_k_padded(K, fp64);
    if (KP < 0)
        return hipErrorInvalidValue;
    if (fp64)
        hipLaunchKernelGGL(k_s_transpose<double>, dim3(256), dim3(256), 0, s, S64, K, W, KP,
                           (double*)St);
    else
        hipLaunchKernelGGL(k_s_transpose<float>, dim3(256), dim3(256), 0, s, S64, K, W, KP,
                           (float*)St);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LGCD phase kernel for segments whose state does not fit in LDS (few long
// segments, or double-precision state at the paper's sizes).  g and Z stay in
// HBM/L2; LDS holds one best key per chunk of 64 extended positions.
//
// Position q of the extended segment is owned by thread q % 512 for the whole
// run, so every global read-modify-write of g and Z is done by one thread and
// needs no synchronisation.  The 64 positions of chunk c = q / 64 are owned by
// the 64 lanes of wave c % 8: a chunk's maximum is a wave reduction.  After an
// update only the chunks that meet the 2W - 1 window are recomputed; the
// segment argmax is then a block reduction over the chunk maxima.
// ---------------------------------------------------------------------------
template <typename G>
struct ChunkBest {
    typename KeyOps<G>::T key;
    G d;
};

// Recompute chunk c (one position per lane): eq. (3) update of the positions
// inside [wlo, whi] (none when the window is empty), then the best candidate
// of the own positions.  Srow is always a valid row block of S; loads are at
// clamped, valid indices and unconditional, their values selected afterwards.
template <typename G>
__device__ __forceinline__ void gm_chunk(int c, int K, int Kr, int W, int off, int Lm,
                                        int Lext, int ext_lo, int b, int64_t L,
                                        G* __restrict__ gs, const double* __restrict__ Zs,
                                        const G* __restrict__ Srow, G delta, int q0,
                                        int wlo, int whi, const G* __restrict__ n2l,
                                        const G* __restrict__ invl,
                                        const G* __restrict__ linvl, G lam,
                                        ChunkBest<G>* __restrict__ cb)
{
    typedef KeyOps<G> KO;
    const int nd = 2 * W - 1;
    const int lane = threadIdx.x & 63;
    const int q = c * 64 + lane;
    const int j = q - off;
    const bool inq = q < Lext;
    const bool upd = inq && q >= wlo && q <= whi;
    const bool own = inq && j >= 0 && j < Lm;
    typename KO::T best = KO::null();
    G bd = (G)0;
    if (upd || own) {
        G* gp = gs + ext_lo + q;
        const double* zp = Zs + b + (j < 0 ? 0 : (j >= Lm ? Lm - 1 : j));
        const int dj = q - q0 + (W - 1);
        const int djc = dj < 0 ? 0 : (dj >= nd ? nd - 1 : dj);
        for (int k0 = 0; k0 < K; k0 += 8) {
            G gv[8], sv[8];
            double zv[8];
#pragma unroll
            for (int c8 = 0; c8 < 8; ++c8) {
                const int k = k0 + c8;
                const int kc = k < K ? k : K - 1;
                const G gl = gp[(int64_t)kc * L];
                const G sl = Srow[(int64_t)kc * nd + djc];
                const double zl = zp[(int64_t)kc * L];
                gv[c8] = k < K ? gl : (G)0;
                sv[c8] = (upd && k < K) ? sl : (G)0;
                zv[c8] = (own && k < K) ? zl : 0.0;
            }
            if (upd) {
#pragma unroll
                for (int c8 = 0; c8 < 8; ++c8) {
                    const int k = k0 + c8;
                    gv[c8] -= sv[c8] * delta;
                    if (k < K)
                        gp[(int64_t)k * L] = gv[c8];
                }
            }
            if (own) {
#pragma unroll
                for (int c8 = 0; c8 < 8; ++c8) {
                    const int k = k0 + c8;
                    if (k < K) {
                        bool zr;
                        const G d = coord_delta<G>(gv[c8], (G)zv[c8], n2l[k], invl[k], linvl[k],
                                                   lam, &zr);
                        const typename KO::T kc = KO::make(fabs(d), (unsigned)(j * Kr + k));
                        const bool bt = KO::better(kc, best);
                        best = KO::select(bt, kc, best);
                        bd = bt ? d : bd;
                    }
                }
            }
        }
    }
    const typename KO::T w = KO::wave_max(best);
    if (KO::same(best, w)) {
        cb[c].key = w;
        cb[c].d = bd;
    }
}

template <typename G>
__global__ void __launch_bounds__(kPhaseThreads)
k_lgcd_phase_gm(PhaseArgs a)
{
    typedef KeyOps<G> KO;
    typedef typename KO::T KeyT;
    constexpr int NT = kPhaseThreads;
    constexpr int NW = NT / 64;
    const int K = a.K;
    const int W = a.W;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;

    const int sid = a.list[blockIdx.x];
    if (a.dirty[sid] == 0)
        return;

    extern __shared__ __align__(16) unsigned char smem[];
    const SegDesc sd = a.segs[sid];
    const int64_t L = sd.L;
    const int b = sd.b;
    const int Lm = sd.e - sd.b;
    const int ext_lo = b - (W - 1) > 0 ? b - (W - 1) : 0;
    const int ext_hi = sd.e + (W - 1) < sd.L ? sd.e + (W - 1) : sd.L;
    const int Lext = ext_hi - ext_lo;
    const int off = b - ext_lo;
    const int nch = (Lext + 63) / 64;

    ChunkBest<G>* cb = reinterpret_cast<ChunkBest<G>*>(smem);        // [nch]
    Slot<G>* slots = reinterpret_cast<Slot<G>*>(cb + a.lext_max / 64 + 1);  // [2][NW]
    G* n2l = reinterpret_cast<G*>(slots + 2 * NW);
    G* invl = n2l + K;
    G* linvl = invl + K;

    G* __restrict__ gs = reinterpret_cast<G*>(a.g) + sd.z_off;
    double* __restrict__ Zs = a.Z + sd.z_off;
    const G* __restrict__ S = reinterpret_cast<const G*>(a.S);  // [K][K][2W-1]
    const G lam = (G)a.sigs[sd.sig].lam;
    const double eps_stop = a.sigs[sd.sig].eps_stop;
    const int nd = 2 * W - 1;
    for (int k = tid; k < K; k += NT) {
        const G iv = reinterpret_cast<const G*>(a.inv_n2)[k];
        n2l[k] = reinterpret_cast<const G*>(a.n2)[k];
        invl[k] = iv;
        linvl[k] = lam * iv;
    }
    __syncthreads();

    for (int c = wave; c < nch; c += NW)
        gm_chunk<G>(c, K, a.K, W, off, Lm, Lext, ext_lo, b, L, gs, Zs, S, (G)0, 0, 0,
                        -1, n2l, invl, linvl, lam, cb);  // empty window: no update
    __syncthreads();

    int it = 0;
    auto argmax = [&](KeyT& out, G& dout) __attribute__((always_inline)) {
        KeyT m = KO::null();
        G d = (G)0;
        for (int c = tid; c < nch; c += NT) {
            const KeyT kc = cb[c].key;
            const bool bt = KO::better(kc, m);
            m = KO::select(bt, kc, m);
            d = bt ? cb[c].d : d;
        }
        KeyT bm[1] = {m};
        G bdl[1] = {d};
        block_argmax<G, 1>(bm, bdl, slots + (it & 1) * NW, out, dout);
        ++it;
    };
    KeyT kb;
    G db;
    argmax(kb, db);

    int n = 0;
    bool conv = false;
    bool touch_l = false, touch_r = false;
    for (;;) {
        if (KO::value(kb) < eps_stop) {
            conv = true;
            break;
        }
        if (n == a.cap)
            break;
        const unsigned kidx = KO::index(kb);
        const int j0 = (int)(kidx / (unsigned)K);
        const int k0 = (int)kidx - j0 * K;
        const int q0 = j0 + off;
        const G delta = db;

        if (tid == (q0 % NT)) {
            double* zp = Zs + (int64_t)k0 * L + b + j0;
            const double zo = *zp;
            bool zr;
            (void)coord_delta<G>(gs[(int64_t)k0 * L + ext_lo + q0], (G)zo, n2l[k0], invl[k0],
                                 linvl[k0],
                                 lam, &zr);
            *zp = zr ? 0.0 : zo + (double)delta;
            if (a.trace) {
                const unsigned long long r = atomicAdd(&a.counters->trace_n, 1ull);
                if ((long long)r < a.trace_cap) {
                    dicod_trace_rec rec;
                    rec.phase = a.phase;
                    rec.seg = sid;
                    rec.k0 = k0;
                    rec.n_local = n;
                    rec.t0 = (int64_t)b + j0;
                    rec.delta = zr ? -zo : (double)delta;
                    a.trace[r] = rec;
                }
            }
        }
        // (the chunk pass below reads this Z entry on the same thread)
        const int wlo = q0 - (W - 1) > 0 ? q0 - (W - 1) : 0;
        const int whi = q0 + (W - 1) < Lext - 1 ? q0 + (W - 1) : Lext - 1;
        if (q0 - (W - 1) < off && sd.left >= 0)
            touch_l = true;
        if (q0 + (W - 1) >= off + Lm && sd.right >= 0)
            touch_r = true;
        const G* __restrict__ Srow = S + (size_t)k0 * K * nd;
        for (int c = wlo / 64 + ((wave - wlo / 64) % NW + NW) % NW; c <= whi / 64; c += NW)
            gm_chunk<G>(c, K, a.K, W, off, Lm, Lext, ext_lo, b, L, gs, Zs, Srow, delta,
                            q0, wlo, whi, n2l, invl, linvl, lam, cb);
        __syncthreads();
        ++n;
        argmax(kb, db);
    }

    if (n > 0 && tid == 0) {
        atomicAdd(&a.phase_upd[(size_t)sd.sig * a.phase_stride + a.phase], (unsigned long long)n);
        atomicAdd(&a.sig_upd[sd.sig], (unsigned long long)n);
        atomicMax(&a.sig_last_upd[sd.sig], a.phase);
        atomicAdd(&a.counters->seg_runs, 1ull);
        if (a.changed)
            a.changed[sid] = 1u;
    }
    if (tid == 0) {
        a.dirty[sid] = conv ? 0u : 1u;
        if (touch_l)
            a.dirty[sd.left] = 1u;
        if (touch_r)
            a.dirty[sd.right] = 1u;
    }
}

size_t lgcd_gm_lds_bytes(int K, int lext_max, bool fp64)
{
    const size_t cbs = fp64 ? sizeof(ChunkBest<double>) : sizeof(ChunkBest<float>);
    const size_t sls = fp64 ? sizeof(Slot<double>) : sizeof(Slot<float>);
    const size_t e = fp64 ? sizeof(double) : sizeof(float);
    return cbs * ((size_t)lext_max / 64 + 1) + sls * 2 * (kPhaseThreads / 64) + 3 * e * (size_t)K;
}

template <typename G>
static hipError_t launch_gm_k(const PhaseArgs& a, size_t lds, hipStream_t s)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_lgcd_phase_gm<G>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_lgcd_phase_gm<G>), dim3((unsigned)a.n_list), dim3(kPhaseThreads),
                       lds, s, a);
    return hipGetLastError();
}

hipError_t launch_lgcd_phase_gm(const PhaseArgs& a, bool fp64, size_t* lds_bytes,
                                hipStream_t s)
{
    if (a.n_list <= 0)
        return hipSuccess;
    const size_t lds = lgcd_gm_lds_bytes(a.K, a.lext_max, fp64);
    if (lds_bytes)
        *lds_bytes = lds;
    if (lds > kLdsBytes)
        return hipErrorInvalidValue;
    if (fp64)
        return launch_gm_k<double>(a, lds, s);
    return launch_gm_k<float>(a, lds, s);
}

// ---------------------------------------------------------------------------
// Double-precision check (final stop test and refresh).
// ---------------------------------------------------------------------------

// Non-zero masks: word w of a signal is bit i = (Z_k[64 b + i] != 0), with
// w = k * ceil(L / 64) + b.  A wave handles kMaskWords consecutive words:
// their signal, atom and block indices are scalar arithmetic (the signal is
// looked up and (k, b) divided out once per wave, then stepped word by word),
// and all their loads are issued before the first ballot.
constexpr int kMaskWords = 16;

__global__ void __launch_bounds__(256)
k_nz_mask(const double* __restrict__ Z, const SigDesc* __restrict__ sig,
          const int64_t* __restrict__ mask_pref, int n_sig, int K, int64_t n_words,
          unsigned long long* __restrict__ masks)
{
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t w0 = ((int64_t)blockIdx.x * 4 + wv) * kMaskWords;
    if (w0 >= n_words)
        return;
    int si = find_sig(mask_pref, n_sig, w0);
    int64_t pref_next = mask_pref[si + 1];
    SigDesc sd = sig[si];
    int64_t nb = (sd.L + 63) / 64;
    int64_t k = (w0 - mask_pref[si]) / nb;   // word w0 = k nb + b of signal si
    int64_t b = (w0 - mask_pref[si]) - k * nb;
    double z[kMaskWords];
#pragma unroll
    for (int i = 0; i < kMaskWords; ++i) {
        const int64_t w = w0 + i;
        z[i] = 0.0;
        if (w >= n_words)
            continue;
        while (w >= pref_next) {  // next signal (every signal has at least one word),
            ++si;                 // entered at its word 0
            pref_next = mask_pref[si + 1];
            sd = sig[si];
            nb = (sd.L + 63) / 64;
            k = 0;
            b = 0;
        }
        const int64_t t = b * 64 + lane;
        const int64_t tc = t < sd.L ? t : sd.L - 1;  // a valid address, selected below
        const double v = Z[sd.z_off + (k < K ? k : K - 1) * sd.L + tc];
        z[i] = (k < K && t < sd.L) ? v : 0.0;
        if (++b == nb) {
            b = 0;
            ++k;
        }
    }
#pragma unroll
    for (int i = 0; i < kMaskWords; ++i) {
        const unsigned long long m = __ballot(z[i] != 0.0);
        if (lane == 0 && w0 + i < n_words)
            masks[w0 + i] = m;
    }
}

hipError_t launch_nz_mask(const double* Z, const SigDesc* sig, const int64_t* mask_pref,
                          int n_sig, int K, int64_t n_words, unsigned long long* masks,
                          hipStream_t s)
{
    if (n_words <= 0)
        return hipSuccess;
    const int64_t blocks = (n_words + 4 * kMaskWords - 1) / (4 * kMaskWords);
    hipLaunchKernelGGL(k_nz_mask, dim3((unsigned)blocks), dim3(256), 0, s, Z, sig, mask_pref,
                       n_sig, K, n_words, masks);
    return hipGetLastError();
}

__device__ __forceinline__ double block_sum256(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max256(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
}

// Atoms of one check block: the block stages kper padded rows of S (2W
// doubles each) per source atom in each of its two LDS buffers; 0 when one
// row does not fit.
int check_atoms_per_block(int K, int W)
{
    const size_t row = (size_t)2 * W * sizeof(double);
    size_t budget = (size_t)24 << 10;  // per buffer: three blocks per CU
    if (row > budget)
        budget = (kLdsBytes - ((size_t)16 << 10)) / 2;
    const int kmax = (int)std::min<size_t>((size_t)kCheckKB, budget / row);
    if (kmax < 1 || K < 1)
        return 0;
    const int nb = (K + kmax - 1) / kmax;
    return (K + nb - 1) / nb;
}

int check_kblocks(int K, int W)
{
    const int kp = check_atoms_per_block(K, W);
    return kp > 0 ? (K + kp - 1) / kp : 0;
}

size_t check_s_elems(int K, int W)
{
    return (size_t)K * K * 2 * W + 128;  // + 1 KB read past the last block by the copies
}

// doubles per LDS stage buffer (whole 1 KB copy chunks)
static int check_stage_stride(int kper, int W)
{
    return (int)((((size_t)kper * 2 * W * sizeof(double) + 1023) / 1024) * 128);
}

constexpr int kCheckList = 448;  // listed non-zeros per pass (LDS)
constexpr int kCheckJ = kCheckSpan / 256;

// Exclusive prefix sum of v over the 256 threads; *total gets the sum.
// All threads call it.
__device__ __forceinline__ int block_scan256(int v, int* total, int* wsum)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        wsum[wave] = x;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        base += w < wave ? wsum[w] : 0;
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// g_k[t] = beta0_k[t] - sum_{l, s} S_{k,l}[t - s] Z_l[s] over the non-zeros of
// Z (eq. (3) summed over every applied update), then in double for every
// coordinate: Delta Z = Sh(g + |D_k|^2 z, lambda) / |D_k|^2 - z, the optimality
// residuals, and the objective partials.  The residual energy follows from g:
// with S Z = D^T (Z * D) and beta0 = D^T X,
//   |X - Z * D|^2 = |X|^2 - 2 <beta0, Z> + <Z, S Z> = |X|^2 - <beta0 + g, Z>.
// A block owns kCheckSpan positions of one signal (thread tid: t_a + tid +
// 256 j) and the atoms [kb, kb + kper).  It lists the non-zeros within reach
// (from the masks, in (l, s) order) in LDS; for each source atom l the rows
// S_{kb.., l}[.] (contiguous in the padded [l][k][2W] copy Sc) are copied
// into one of two LDS buffers by direct global-to-LDS loads, the next atom's
// copy in flight while the current one is summed.  The sums run over (l, s)
// in increasing order.  With g_in the maintained double state is checked as
// it is.  part per (y-block, tile): max|dz|, kkt_on, kkt_off, l1, max|z|, nnz,
// |X|^2 (y-block 0 only), <beta0 + g, Z>.  KB >= kper atoms are summed
// without branches (rows past the block's last atom repeat it; their sums
// are never read).
template <int J, int KB>
__global__ void __launch_bounds__(256)
k_grad_check(const float* __restrict__ X, const double* __restrict__ beta0,
             const double* __restrict__ Z, const unsigned long long* __restrict__ masks,
             const double* __restrict__ Sc, const double* __restrict__ n2v, int K, int P,
             int W, int kper, const SigDesc* __restrict__ sig,
             const int64_t* __restrict__ tile_pref, int n_sig, double flag_eps,
             const uint32_t* __restrict__ sig_done, uint32_t* __restrict__ dirty,
             float* __restrict__ g32, double* __restrict__ g64,
             const double* __restrict__ g_in, double* __restrict__ part,
             float* __restrict__ z32, const uint32_t* __restrict__ changed)
{
    extern __shared__ __align__(16) double sst[];  // 2 x [kper][2W]: S_{kb+k,l}[d - W + 1]
    __shared__ int ls[kCheckList];                 // listed non-zeros (l, s, Z_l[s])
    __shared__ int lk[kCheckList];
    __shared__ double lz[kCheckList];
    __shared__ int wsum[4];
    __shared__ double red[4];
    const int nd = 2 * W - 1;
    const int ndp = 2 * W;  // padded row: 16-byte multiple
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t tile = blockIdx.x;
    const int si = find_sig(tile_pref, n_sig, tile);
    const SigDesc sd = sig[si];
    const int64_t L = sd.L;
    const int64_t t_a = (tile - tile_pref[si]) * (int64_t)(256 * J);
    const int kb = blockIdx.y * kper;
    const int kn = K - kb < kper ? K - kb : kper;
    const double* __restrict__ Zs = Z + sd.z_off;
    // accepted signals are only measured: no refresh, no new dirty segments
    const bool frozen = sig_done && sig_done[si] != 0u;

    // With change flags: a tile none of whose reach [t_a - W + 1,
    // t_a + span + W - 1) lies in a segment whose Z changed since the last
    // check keeps its partials and its refreshed state from that check; it
    // only marks its segments dirty again when its largest |Delta Z| still
    // reaches flag_eps.
    if (changed) {
        const int64_t lo = t_a - (W - 1) > 0 ? t_a - (W - 1) : 0;
        const int64_t hi = t_a + 256 * J + (W - 1) < L ? t_a + 256 * J + (W - 1) : L;
        const int64_t m0 = ((lo + 1) * (int64_t)sd.M - 1) / L;
        const int64_t m1 = (hi * (int64_t)sd.M - 1) / L;
        bool any = false;
        for (int64_t m = m0; m <= m1; ++m)
            any = any || changed[sd.seg_base + m] != 0u;
        if (!any) {
            const double* o = part + ((int64_t)blockIdx.y * gridDim.x + tile) * kCheckParts;
            if (tid == 0 && dirty && !frozen && o[0] >= flag_eps) {
                const int64_t e = t_a + 256 * J < L ? t_a + 256 * J : L;
                const int64_t q0 = ((t_a + 1) * (int64_t)sd.M - 1) / L;
                const int64_t q1 = (e * (int64_t)sd.M - 1) / L;
                for (int64_t m = q0; m <= q1; ++m)
                    dirty[sd.seg_base + m] = 1u;
            }
            return;
        }
    }

    // loads at clamped (valid) indices, unconditional so that they are all in
    // flight together; the values past the ends are never used
    double acc[J][KB];
    {
        const double* __restrict__ a0 = (g_in ? g_in : beta0) + sd.z_off;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int64_t t = t_a + tid + 256 * j;
            const int64_t tc = t < L ? t : L - 1;
#pragma unroll
            for (int k = 0; k < KB; ++k)
                acc[j][k] = a0[(int64_t)(kb + (k < kn ? k : kn - 1)) * L + tc];
        }
    }

    if (!g_in) {
        const int bstride = (int)(((size_t)kper * ndp * sizeof(double) + 1023) / 1024 * 128);
        const int nch = (kn * ndp * (int)sizeof(double) + 1023) >> 10;  // 1 KB copy chunks
        // rows of atom l into buffer buf: 64 lanes x 16 bytes per wave and chunk
        auto stage = [&](int l, int buf) __attribute__((always_inline)) {
            const char* src = reinterpret_cast<const char*>(Sc + ((int64_t)l * K + kb) * ndp) +
                              lane * 16;
            char* dst = reinterpret_cast<char*>(sst + (size_t)buf * bstride);
            for (int c = wave; c < nch; c += 4)
                __builtin_amdgcn_global_load_lds(
                    (const void*)(src + (size_t)c * 1024),
                    (__attribute__((address_space(3))) void*)(dst + (size_t)c * 1024), 16, 0,
                    0);
        };
        const int64_t s_lo = t_a - (W - 1) > 0 ? t_a - (W - 1) : 0;
        const int64_t s_hi = t_a + 256 * J + (W - 1) < L ? t_a + 256 * J + (W - 1) : L;
        const int64_t nbk = (L + 63) / 64;
        const int64_t b_lo = s_lo >> 6;
        const int nbw = (int)(((s_hi - 1) >> 6) - b_lo + 1);
        const int items = K * nbw;  // mask words in reach, atom-major
        const unsigned long long* __restrict__ msk = masks + sd.nz_off;
        // row offsets of the block's atoms in a buffer (past the last atom: its row)
        int rowoff[KB];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
            rowoff[kk] = (kk < kn ? kk : kn - 1) * ndp;
        const int n_own = L - t_a < 256 * J ? (int)(L - t_a) : 256 * J;  // positions in the tile
        int cur_l = -1, cb = 0;  // atom whose rows sit in buffer cb
        int staged_l = -1;       // atom whose copy into buffer cb ^ 1 is in flight
        for (int i0 = 0; i0 < items; i0 += 256) {
            const int it = i0 + tid;
            unsigned long long m = 0ull;
            int k = 0;
            int64_t pos0 = 0;
            if (it < items) {
                k = it / nbw;
                const int64_t bb = b_lo + (it - k * nbw);
                pos0 = bb * 64;
                m = msk[(int64_t)k * nbk + bb];
                if (pos0 < s_lo)
                    m &= ~0ull << (int)(s_lo - pos0);
                if (pos0 + 64 > s_hi)
                    m &= (1ull << (int)(s_hi - pos0)) - 1ull;  // s_hi - pos0 in [1, 63]
            }
            const int cm = __popcll(m);
            int tot;
            const int off = block_scan256(cm, &tot, wsum);
            for (int base = 0; base < tot; base += kCheckList) {
                // list entries [base, base + kCheckList) of this round
                if (cm > 0 && off < base + kCheckList && off + cm > base) {
                    unsigned long long mm = m;
                    int idx = off;
                    while (mm && idx < base + kCheckList) {
                        const int bit = __ffsll(mm) - 1;
                        mm &= mm - 1ull;
                        if (idx >= base) {
                            const int sp = (int)(pos0 + bit);
                            ls[idx - base] = sp;
                            lk[idx - base] = k;
                            lz[idx - base] = Zs[(int64_t)k * L + sp];
                        }
                        ++idx;
                    }
                }
                lds_barrier();
                const int cnt = tot - base < kCheckList ? tot - base : kCheckList;
                int e = 0;
                while (e < cnt) {
                    const int l = lk[e];
                    int e1 = e + 1;
                    while (e1 < cnt && lk[e1] == l)
                        ++e1;
                    if (l != cur_l) {
                        if (staged_l != l)
                            stage(l, cb ^ 1);  // not copied ahead
                        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's copies landed
                        lds_barrier();  // every copy landed; the previous rows are consumed
                        cb ^= 1;
                        cur_l = l;
                        staged_l = -1;
                        if (e1 < cnt) {
                            staged_l = lk[e1];
                            stage(staged_l, cb ^ 1);  // in flight during this atom's sums
                        }
                    }
                    const double* __restrict__ rows = sst + (size_t)cb * bstride + tid;
                    // up to 64 non-zeros of this atom at a time, one per lane:
                    // lane c holds the lag base d0 (lag of position t_a + tid +
                    // 256 j is d0 + tid + 256 j; 32-bit, positions are below
                    // 2^31) and the value of non-zero c0 + c.  Per strip j a
                    // ballot marks the non-zeros whose lags for this wave's 64
                    // positions meet [0, nd); the wave then walks those bits in
                    // increasing order (the order of the list, so every sum
                    // keeps the order of (l, s)), reading d0 and z from their
                    // lanes.
                    for (int c0 = e; c0 < e1; c0 += 64) {
                        const bool have = lane < e1 - c0;
                        const int my_d0 = have ? (int)(t_a - ls[c0 + lane]) + (W - 1) : -(1 << 29);
                        const double my_z = have ? lz[c0 + lane] : 0.0;
                        const long long zbits = __double_as_longlong(my_z);
#pragma unroll
                        for (int j = 0; j < J; ++j) {
                            const int dw = my_d0 + wave * 64 + 256 * j;
                            unsigned long long m = __ballot(have && dw + 63 >= 0 && dw < nd);
                            while (m) {
                                const int c = __builtin_ctzll(m);
                                m &= ~(1ull << c);
                                const int d0 = __builtin_amdgcn_readlane(my_d0, c);
                                const unsigned zlo = (unsigned)__builtin_amdgcn_readlane(
                                    (int)(unsigned)zbits, c);
                                const unsigned zhi = (unsigned)__builtin_amdgcn_readlane(
                                    (int)(zbits >> 32), c);
                                const double z = __longlong_as_double(
                                    (long long)(((unsigned long long)zhi << 32) | zlo));
                                const int d = d0 + tid + 256 * j;
                                if ((unsigned)d < (unsigned)nd && tid + 256 * j < n_own) {
                                    const double* __restrict__ sr = rows + (d0 + 256 * j);
                                    double sv[KB];
#pragma unroll
                                    for (int kk = 0; kk < KB; ++kk)
                                        sv[kk] = sr[rowoff[kk]];
#pragma unroll
                                    for (int kk = 0; kk < KB; ++kk)
                                        acc[j][kk] -= sv[kk] * z;
                                }
                            }
                        }
                    }
                    e = e1;
                }
                lds_barrier();  // the list is consumed
            }
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);  // no copy left in flight at exit
    }

    double mdz = 0.0, kon = 0.0, koff = 0.0, l1 = 0.0, mz = 0.0, nnz = 0.0, x2 = 0.0, bz = 0.0;
    double bx = 0.0, gm = 0.0;
    const double lam = sd.lam;
    // 1 / |D_k|^2 once per atom: the per-coordinate quotients below become
    // products (within an ulp of the quotient; a double division is some
    // twenty instructions, and every zero coordinate needs one)
    double inv[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k)
        inv[k] = 1.0 / n2v[kb + (k < kn ? k : kn - 1)];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int64_t t = t_a + tid + 256 * j;
        double zv[KB];
        {
            const int64_t tc = t < L ? t : L - 1;
#pragma unroll
            for (int k = 0; k < KB; ++k)
                zv[k] = Zs[(int64_t)(kb + (k < kn ? k : kn - 1)) * L + tc];
        }
        if (t >= L)
            continue;
        bool flag = false;
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            if (k >= kn)
                continue;
            const int kk = kb + k;
            const int64_t o = sd.z_off + (int64_t)kk * L + t;
            const double z = zv[k];
            const double n2 = n2v[kk];
            const double g = acc[j][k];
            const double bb = g + n2 * z;
            const double ab = fabs(bb) - lam;
            const double zp = ab > 0.0 ? (bb > 0.0 ? ab : -ab) * inv[k] : 0.0;
            const double dz = fabs(zp - z);
            mdz = fmax(mdz, dz);
            gm = fmax(gm, fabs(g));
            if (dz >= flag_eps)
                flag = true;
            if (z != 0.0) {
                kon = fmax(kon, fabs(g - (z > 0.0 ? lam : -lam)) * inv[k]);
                l1 += fabs(z);
                mz = fmax(mz, fabs(z));
                nnz += 1.0;
                const double b0 = beta0[o];
                bz += (b0 + g) * z;
                bx += b0 * z;
            } else {
                koff = fmax(koff, fmax(fabs(g) - lam, 0.0) * inv[k]);
            }
            if (g32 && !frozen)
                g32[o] = (float)g;
            if (z32 && !frozen)
                z32[o] = (float)z;
            if (g64 && !frozen)
                g64[o] = g;
        }
        if (flag && dirty && !frozen) {
            // segment m holds t iff floor(m L / M) <= t < floor((m+1) L / M)
            const int64_t m = ((t + 1) * (int64_t)sd.M - 1) / L;
            dirty[sd.seg_base + m] = 1u;
        }
    }
    if (blockIdx.y == 0) {
        // |X|^2 over the samples [t_a, t_a + span); the last tile of a signal
        // also takes the final W - 1 samples
        const int64_t u_hi = t_a + 256 * J >= L ? sd.T : t_a + 256 * J;
        for (int64_t u = t_a + tid; u < u_hi; u += 256)
            for (int p = 0; p < P; ++p) {
                const double x = (double)X[sd.x_off + (int64_t)p * sd.T + u];
                x2 += x * x;
            }
    }
    mdz = block_max256(mdz, red);
    kon = block_max256(kon, red);
    koff = block_max256(koff, red);
    l1 = block_sum256(l1, red);
    mz = block_max256(mz, red);
    nnz = block_sum256(nnz, red);
    x2 = block_sum256(x2, red);
    bz = block_sum256(bz, red);
    bx = block_sum256(bx, red);
    gm = block_max256(gm, red);
    if (tid == 0) {
        double* o = part + ((int64_t)blockIdx.y * gridDim.x + tile) * kCheckParts;
        o[0] = mdz;
        o[1] = kon;
        o[2] = koff;
        o[3] = l1;
        o[4] = mz;
        o[5] = nnz;
        o[6] = x2;
        o[7] = bz;
        o[8] = bx;
        o[9] = gm;
    }
}

hipError_t launch_grad_check(const float* X, const double* beta0, const double* Z,
                             const unsigned long long* masks, const double* Sc,
                             const double* n2, int K, int P, int W, const SigDesc* sig,
                             const int64_t* tile_pref, int n_sig, int64_t n_tiles,
                             double flag_eps, const uint32_t* sig_done, uint32_t* dirty,
                             void* g_state, bool state_fp64, const double* g_in,
                             double* part, float* z32, const uint32_t* changed, hipStream_t s)
{
    const int kper = check_atoms_per_block(K, W);
    if (kper < 1)
        return hipErrorInvalidValue;
    if (n_tiles <= 0)
        return hipSuccess;
    const size_t lds = 2 * (size_t)check_stage_stride(kper, W) * sizeof(double);
    dim3 grid((unsigned)n_tiles, (unsigned)((K + kper - 1) / kper));
    float* g32 = state_fp64 ? (float*)nullptr : (float*)g_state;
    double* g64 = state_fp64 ? (double*)g_state : (double*)nullptr;
    auto go = [&](auto kern) {
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, X, beta0, Z, masks, Sc, n2, K, P, W,
                           kper, sig, tile_pref, n_sig, flag_eps, sig_done, dirty, g32, g64,
                           g_in, part, z32, changed);
        return hipGetLastError();
    };
    static_assert(kCheckKB == 8, "instantiated atom counts");
    if (kper <= 2)
        return go(k_grad_check<kCheckJ, 2>);
    if (kper <= 4)
        return go(k_grad_check<kCheckJ, 4>);
    if (kper <= 7)
        return go(k_grad_check<kCheckJ, 7>);
    return go(k_grad_check<kCheckJ, 8>);
}

// One workgroup per signal reduces its tiles' partials in a fixed order.
__global__ void __launch_bounds__(256)
k_check_reduce(const double* __restrict__ part, const int64_t* __restrict__ pref,
               int64_t n_tiles, int n_kblk, CheckResult* __restrict__ out)
{
    __shared__ double red[4];
    const int si = blockIdx.x;
    double mdz = 0.0, kon = 0.0, koff = 0.0, l1 = 0.0, mz = 0.0, nnz = 0.0, x2 = 0.0, bz = 0.0;
    double bx = 0.0, gm = 0.0;
    for (int kbk = 0; kbk < n_kblk; ++kbk)
        for (int64_t i = pref[si] + threadIdx.x; i < pref[si + 1]; i += 256) {
            const double* p = part + ((int64_t)kbk * n_tiles + i) * kCheckParts;
            mdz = fmax(mdz, p[0]);
            kon = fmax(kon, p[1]);
            koff = fmax(koff, p[2]);
            l1 += p[3];
            mz = fmax(mz, p[4]);
            nnz += p[5];
            x2 += p[6];
            bz += p[7];
            bx += p[8];
            gm = fmax(gm, p[9]);
        }
    mdz = block_max256(mdz, red);
    kon = block_max256(kon, red);
    koff = block_max256(koff, red);
    l1 = block_sum256(l1, red);
    mz = block_max256(mz, red);
    nnz = block_sum256(nnz, red);
    x2 = block_sum256(x2, red);
    bz = block_sum256(bz, red);
    bx = block_sum256(bx, red);
    gm = block_max256(gm, red);
    if (threadIdx.x == 0) {
        CheckResult c;
        c.max_dz = mdz;
        c.kkt_on = kon;
        c.kkt_off = koff;
        c.l1 = l1;
        c.sum_r2 = fmax(x2 - bz, 0.0);  // rounding could leave an exact fit just below 0
        c.max_abs_z = mz;
        c.nnz = nnz;
        c.bx = bx;
        c.gmax = gm;
        c.x2 = x2;
        c.pad = 0.0;
        out[si] = c;
    }
}

hipError_t launch_check_reduce(const double* part, const int64_t* tile_pref, int64_t n_tiles,
                               int n_kblk, int n_sig, CheckResult* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_reduce, dim3((unsigned)n_sig), dim3(256), 0, s, part, tile_pref,
                       n_tiles, n_kblk, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Serving helpers: lambda of newly admitted signals, per-signal phase rings.
// ---------------------------------------------------------------------------
__global__ void k_apply_lambda(SigDesc* tab, const int* slots, const double* lam_in,
                               const unsigned long long* lmax_bits, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double lam = lam_in[i];
    if (lam < 0.0) {
        lam = -lam * __longlong_as_double((long long)lmax_bits[i]);
        if (!(lam > 0.0))
            lam = 1e-300;  // X orthogonal to every atom: Z = 0
    }
    tab[slots[i]].lam = lam;
}

hipError_t launch_apply_lambda(SigDesc* tab, const int* slots, const double* lam_in,
                               const unsigned long long* lmax_bits, int n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_apply_lambda, dim3((n + 255) / 256), dim3(256), 0, s, tab, slots,
                       lam_in, lmax_bits, n);
    return hipGetLastError();
}

__global__ void k_set_eps_stop(SigDesc* tab, int n, double eps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        tab[i].eps_stop = eps;
}

hipError_t launch_set_eps_stop(SigDesc* tab, int n, double eps, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_set_eps_stop, dim3((n + 255) / 256), dim3(256), 0, s, tab, n, eps);
    return hipGetLastError();
}

// dirty[s] = 0 for the segments of signals whose stop test has held: an
// accepted signal's Z is final, whatever its last check flagged.
__global__ void k_clear_done_dirty(const SegDesc* __restrict__ segs, int n_seg,
                                   const uint32_t* __restrict__ done, uint32_t* dirty)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_seg && done[segs[i].sig] != 0u)
        dirty[i] = 0u;
}

hipError_t launch_clear_done_dirty(const SegDesc* segs, int n_seg, const uint32_t* done,
                                   uint32_t* dirty, hipStream_t s)
{
    if (n_seg <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_clear_done_dirty, dim3((n_seg + 255) / 256), dim3(256), 0, s, segs,
                       n_seg, done, dirty);
    return hipGetLastError();
}

__global__ void k_clear_ring(unsigned long long* ring, int rows, int H, int start, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * n)
        return;
    const int r = i / n;
    const int c = i - r * n;
    ring[(size_t)r * H + (start + c) % H] = 0ull;
}

hipError_t launch_clear_ring(unsigned long long* ring, int rows, int H, int start, int n,
                             hipStream_t s)
{
    if (rows <= 0 || n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_clear_ring, dim3((rows * n + 255) / 256), dim3(256), 0, s, ring, rows,
                       H, start, n);
    return hipGetLastError();
}

}  // namespace dicod
