// Device helpers shared by the register-state phase kernels (coloured
// schedule and free-running schedule): vector type, wave reductions, the
// candidate Delta Z of eq. (pb_coord) and the 32-bit argmax key.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dicod {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWaveRecs = 64;  // updates per run at most (mailbox capacity)

struct WSlot {
    unsigned key;
    int pos;
    float delta;
    int pad;
};

// Wave-wide maximum of an unsigned key with DPP row operations: quad
// permutations, half-row and row mirrors, then the row broadcasts of lanes 15
// and 31; lane 63 ends with the maximum, read into a scalar register.
template <int CTRL, int RM>
__device__ __forceinline__ unsigned dpp_max_step(unsigned a)
{
    // lanes the row mask leaves out read 0, the identity of the maximum, so
    // that the move folds into one v_max_u32 with a DPP source
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, CTRL, RM, 0xf, false);
    return o > a ? o : a;
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned a)
{
    a = dpp_max_step<0xB1, 0xf>(a);   // quad_perm [1,0,3,2]
    a = dpp_max_step<0x4E, 0xf>(a);   // quad_perm [2,3,0,1]
    a = dpp_max_step<0x141, 0xf>(a);  // row_half_mirror
    a = dpp_max_step<0x140, 0xf>(a);  // row_mirror
    a = dpp_max_step<0x142, 0xa>(a);  // row_bcast:15 into rows 1 and 3
    a = dpp_max_step<0x143, 0xc>(a);  // row_bcast:31 into rows 2 and 3
    return __builtin_amdgcn_readlane(a, 63);
}

// Lowest lane whose predicate holds (the predicate holds in at least one lane).
__device__ __forceinline__ int first_lane(bool p)
{
    const unsigned long long m = __ballot(p);
    return __builtin_ctzll(m);
}

// v[k] of a register array for a wave-uniform k: a binary search on k, so
// the branches are scalar and only one selection executes.
template <int LO, int HI, int KQ>
__device__ __forceinline__ float pick(const f4 (&v)[KQ], int k)
{
    if constexpr (HI - LO == 1) {
        return v[LO / 4][LO % 4];
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (k < MID)
            return pick<LO, MID, KQ>(v, k);
        return pick<MID, HI, KQ>(v, k);
    }
}

// Delta Z of one coordinate in g-form: beta = g + |D_k|^2 z; Z' = 0 where
// |beta| <= lambda, so Delta Z = -z exactly (the change Z receives); else
// Delta Z = (g - lambda sign(beta)) / |D_k|^2 (eq. (pb_coord)), formed without
// cancellation against z and exact in the subtraction when g is close to
// +-lambda.
__device__ __forceinline__ float cand(float g, float z, float n2, float inv, float lam)
{
    const float bb = fmaf(n2, z, g);
    return fabsf(bb) <= lam ? -z : (g - copysignf(lam, bb)) * inv;
}

__device__ __forceinline__ unsigned make_key(float d, int k)
{
    return (__float_as_uint(d) & 0x7fffffe0u) | (unsigned)(31 - k);
}

__device__ __forceinline__ float key_value(unsigned key)
{
    return __uint_as_float(key & 0x7fffffe0u);
}

// Key of one coordinate: |Delta Z| of cand() with the atom in the low bits.
__device__ __forceinline__ unsigned cand_key(float g, float z, float n2, float inv, float lam,
                                             int k)
{
    return make_key(cand(g, z, n2, inv, lam), k);
}

// Best key over the own position's atoms.  z: this thread's column of the
// LDS array [KQ][threads].  KL atoms of the last group of four are real (the
// rest pad the group and are skipped).  (Two other forms of the soft
// threshold measured slower here than the compare-and-select of cand(): a
// clamp of beta, and the median of g - lambda, g + lambda and -|D_k|^2 z,
// which needs no beta and one instruction less.)
template <int KQ, int KL, int NT>
__device__ __forceinline__ unsigned best_key(const f4 (&g)[KQ], const f4* __restrict__ z,
                                             const f4* __restrict__ cn2,
                                             const f4* __restrict__ cinv, float lam)
{
    unsigned best = 0u;
#pragma unroll
    for (int i = 0; i < KQ; ++i) {
        const f4 n2 = cn2[i], iv = cinv[i];
        const f4 zv = z[i * NT];
#pragma unroll
        for (int c = 0; c < (i == KQ - 1 ? KL : 4); ++c) {
            const unsigned key = cand_key(g[i][c], zv[c], n2[c], iv[c], lam, 4 * i + c);
            best = key > best ? key : best;
        }
    }
    return best;
}

// Real atoms in the last of KQ groups of four when K fills all but that
// group's tail, else 4 (the padded atoms are then carried as zeros).
inline int wave_last_group(int K, int KQ)
{
    const int r = K - 4 * (KQ - 1);
    return r >= 1 && r <= 4 ? r : 4;
}

// g -= s delta over the real atoms.
template <int KQ, int KL>
__device__ __forceinline__ void axpy_state(f4 (&g)[KQ], const f4 (&s)[KQ], float delta)
{
#pragma unroll
    for (int i = 0; i < KQ - 1; ++i)
        g[i] -= s[i] * delta;
#pragma unroll
    for (int c = 0; c < KL; ++c)
        g[KQ - 1][c] -= s[KQ - 1][c] * delta;
}

}  // namespace
}  // namespace dicod
