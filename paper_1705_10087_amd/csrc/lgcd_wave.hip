// Register-state LGCD phase kernel for float state (gfx950).
//
// One segment run is Algorithm 3 restricted to the segment C_m (Sec. 2.2):
// repeat { for every coordinate of the segment, Z' = Sh(beta, lambda) /
// |D_k|^2 (eq. (pb_coord)); take the coordinate with the largest
// |Delta Z| = |Z' - Z|; apply it and the eq. (3) update of beta over the
// 2W - 1 window } until the largest |Delta Z| is below the stop threshold or
// the run has made `cap` updates.
//
// Layout.  A team of TW waves (TW = 1, 2 or 4) runs one segment of at most
// 64 TW positions; thread j of the team owns segment position j and keeps its
// K coefficients of the descent state g = beta - |D_k|^2 Z (g-form: eq. (3)
// then applies uniformly, also at the updated coordinate) in vector
// registers, in groups of four atoms, and its K values of Z (float) in its own
// column of an LDS array (only the updated coordinate's changes).  In an
// update the owner of every position in the window loads its row of the
// correlation table S_{., k0}[t - t0] (St[k0][d][k], 16-byte vectors, the
// rows of consecutive positions are contiguous) and applies g -= S delta to
// its own registers, then re-evaluates its own candidates.
//
// Argmax.  A candidate is one 32-bit key: the bits of |Delta Z| with the low
// five mantissa bits replaced by 31 - k, so an unsigned maximum over keys
// picks the largest |Delta Z| (to 2^-18 relative) and, among equal values, the
// smallest atom.  The team maximum is a DPP reduction inside each wave; the
// winning lane is the lowest lane holding the maximum (smallest position).
// With TW = 1 a segment is one wave and an update needs no barrier at all;
// with TW > 1 the waves exchange (key, lane, delta) through LDS slots with
// one barrier per update (slots double-buffered by update parity).  The
// applied change delta is recomputed exactly from the winner's registers.
//
// Boundary.  An update whose window reaches a neighbouring segment (the
// W - 1 positions next to the edge) is sent to that neighbour as a record
// (k0, t0, delta) in its mailbox in HBM -- the message of Algorithm 2 -- and
// the neighbour applies its records, from the left neighbour first, each in
// the order sent, when it next runs, before it picks a coordinate.  Under the
// coloured schedule a segment that receives records is marked dirty and runs
// before the sender runs again, so a mailbox holds at most one run's records,
// and the result equals applying the records at once (up to the order of the
// float additions).  A run therefore moves only its own state through HBM.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "dicod_internal.h"
#include "lgcd_wave_util.h"

namespace dicod {
namespace {

// Occupancy: the kernel is bound by the latency of its per-update chain
// (argmax, S-row loads, window update), which more resident waves hide.  The
// register budget asks for the waves the LDS footprint allows: four per SIMD
// for one-wave teams (four segments of 28 KB of z per workgroup), five for
// larger teams (up to 96 registers), one less for 32 atoms.  Without a cap the
// compiler spends up to 131 registers and three waves remain.  The S rows of
// an update are pinned in flight together by a scheduling barrier: under the
// register cap the scheduler would otherwise reuse one register quad and wait
// for each row in turn (measured 15-30% slower).
template <int KQ, int KL, int TW>
__global__ void __launch_bounds__(TW == 2 ? 128 : 256)
__attribute__((amdgpu_waves_per_eu(KQ == 8 ? (TW == 1 ? 3 : 4) : (TW == 1 ? 4 : 5))))
k_lgcd_wave(PhaseArgs a)
{
    constexpr int SPB = TW == 1 ? 4 : 1;      // segments per workgroup
    constexpr int NTT = 64 * TW;              // threads per team (one segment)
    constexpr int KP = 4 * KQ;
    const int lane = threadIdx.x & 63;
    // uniform in the wave: the segment's descriptor and pointers then live in
    // scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int team = TW == 1 ? wave : 0;
    const int tt = TW == 1 ? lane : (int)threadIdx.x;  // position owned in the segment

    constexpr int NT = SPB * NTT;             // threads per workgroup
    __shared__ f4 s_cst[SPB][2][KQ];            // |D_k|^2 and 1 / |D_k|^2
    __shared__ f4 s_u[KQ * NT];                 // Z in float: [atom group][thread]
    __shared__ WSlot s_slot[2][TW];
    __shared__ BoundaryRec s_in[SPB][2 * kWaveRecs];  // records received
    f4* __restrict__ u = s_u + threadIdx.x;    // this thread's column (stride NT)

    const int li = blockIdx.x * SPB + team;
    if (li >= a.n_list)
        return;
    const int sid = a.list[li];
    if (a.dirty[sid] == 0)
        return;

    const SegDesc sd = a.segs[sid];
    const int K = a.K;
    const int W = a.W;
    const int nd = 2 * W - 1;
    const int64_t L = sd.L;
    const int b = sd.b;
    const int Lm = sd.e - sd.b;
    float* __restrict__ gs = reinterpret_cast<float*>(a.g) + sd.z_off;
    double* __restrict__ Zs = a.Z + sd.z_off;
    float* __restrict__ zs32 = a.z32 + sd.z_off;
    const float* __restrict__ St = reinterpret_cast<const float*>(a.S);  // [K][nd][KP]
    const float lam = (float)a.sigs[sd.sig].lam;
    const float eps_stop = (float)a.sigs[sd.sig].eps_stop;

    // per-atom constants of this team (padded atoms: |D|^2 = 1; their g and
    // u are 0, so their candidate is 0)
    // (scalar stores: each thread writes its own atoms' words, never a whole
    // 16-byte vector, which would be a read-modify-write racing with the
    // threads writing the vector's other words)
    f4* cn2 = s_cst[team][0];
    f4* cinv = s_cst[team][1];
    for (int k = tt; k < KP; k += NTT) {
        reinterpret_cast<float*>(cn2)[k] = k < K ? reinterpret_cast<const float*>(a.n2)[k] : 1.0f;
        reinterpret_cast<float*>(cinv)[k] =
            k < K ? reinterpret_cast<const float*>(a.inv_n2)[k] : 1.0f;
    }
    if (TW > 1)
        __syncthreads();
    else
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

    // own state: g and u = |D_k|^2 Z of position j = tt.  Every lane loads
    // (idle lanes at position 0: their values are never used) and padded atoms
    // load atom K - 1 and are zeroed by a uniform select, so that the loads
    // are unconditional and all in flight at once.
    const bool own = tt < Lm;
    const int jc = own ? tt : 0;
    f4 g[KQ], uz[KQ];
    {
        const float* pg = gs + b + jc;
        const float* pz = zs32 + b + jc;
#pragma unroll
        for (int i = 0; i < KQ; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                g[i][c] = *pg;
                uz[i][c] = *pz;
                if (4 * i + c + 1 < K) {  // padded atoms reread atom K - 1
                    pg += L;
                    pz += L;
                }
            }
    }
    // mailbox counts: the records waiting for this segment, and where this
    // run's records to the neighbours start (their boxes are emptied when they
    // run, which under the coloured schedule is before this segment runs again)
    uint32_t* __restrict__ bn = a.box_n;
    const uint32_t in_l = bn[(size_t)sid * 2 + 0], in_r = bn[(size_t)sid * 2 + 1];
    const uint32_t base_l = sd.left >= 0 ? bn[(size_t)sd.left * 2 + 1] : 0u;
    const uint32_t base_r = sd.right >= 0 ? bn[(size_t)sd.right * 2 + 0] : 0u;
#pragma unroll
    for (int i = 0; i < KQ; ++i) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const bool pad = 4 * i + c >= K;
            g[i][c] = pad ? 0.0f : g[i][c];
            uz[i][c] = pad ? 0.0f : uz[i][c];
        }
        u[i * NT] = uz[i];
    }
    int tlo = INT_MAX, thi = -1;  // own positions whose g changed (written back)
    // records of the neighbours' last runs, from the left neighbour, then from
    // the right one, each in the order sent: staged in LDS with one load per
    // record, then applied one at a time (a record out of a position's reach
    // reads a valid row and applies a zero change)
    const int n_in = (int)(in_l + in_r);
    BoundaryRec* rin = s_in[team];
    for (int i = tt; i < n_in; i += NTT)
        rin[i] = i < (int)in_l ? a.box[((size_t)sid * 2 + 0) * a.box_cap + i]
                               : a.box[((size_t)sid * 2 + 1) * a.box_cap + (i - (int)in_l)];
    if (TW > 1)
        __syncthreads();
    else
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int r = 0; r < n_in; ++r) {
        const BoundaryRec r0 = rin[r];
        const int j0a = r0.t0 - b;
        const int lo_a = j0a - (W - 1) > 0 ? j0a - (W - 1) : 0;
        const int hi_a = j0a + (W - 1) < Lm - 1 ? j0a + (W - 1) : Lm - 1;
        tlo = lo_a < tlo ? lo_a : tlo;
        thi = hi_a > thi ? hi_a : thi;
        const int da = tt - j0a + (W - 1);
        const bool ina = own && da >= 0 && da < nd;
        const f4* sa = reinterpret_cast<const f4*>(
            St + ((size_t)r0.k0 * nd + (ina ? da : 0)) * KP);
        f4 va[KQ];
#pragma unroll
        for (int i = 0; i < KQ; ++i)
            va[i] = sa[i];
        __builtin_amdgcn_sched_barrier(0);  // the row in flight at once
        axpy_state<KQ, KL>(g, va, ina ? r0.delta : 0.0f);
    }

    // team argmax: key, position and exact change delta of the best candidate
    int it = 0;
    auto argmax = [&](unsigned mine, unsigned& kb, int& j0, float& db) __attribute__((always_inline)) {
        const unsigned wk = wave_max_u32(mine);
        const int wl = first_lane(mine == wk);
        const int k0w = 31 - (int)(wk & 31u);
        const int kk = k0w < KP ? k0w : 0;
        // exact delta of the wave's winner, from its registers and u column
        const float gw = __int_as_float(
            __builtin_amdgcn_readlane(__float_as_int(pick<0, KP, KQ>(g, kk)), wl));
        const float zw = s_u[(kk / 4) * NT + (threadIdx.x - lane) + wl][kk % 4];
        const float dw = cand(gw, zw, cn2[kk / 4][kk % 4], cinv[kk / 4][kk % 4], lam);
        if (TW == 1) {
            kb = wk;
            j0 = wl;
            db = dw;
        } else {
            WSlot* sl = s_slot[it & 1];
            if (lane == 0) {
                WSlot w;
                w.key = wk;
                w.pos = wave * 64 + wl;
                w.delta = dw;
                w.pad = 0;
                sl[wave] = w;
            }
            __syncthreads();
            WSlot bst = sl[0];
#pragma unroll
            for (int v = 1; v < TW; ++v) {
                const WSlot o = sl[v];
                if (o.key > bst.key)
                    bst = o;
            }
            kb = (unsigned)__builtin_amdgcn_readfirstlane((int)bst.key);
            j0 = __builtin_amdgcn_readfirstlane(bst.pos);
            db = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(bst.delta)));
        }
        ++it;
    };

    unsigned mine = own ? best_key<KQ, KL, NT>(g, u, cn2, cinv, lam) : 0u;
    unsigned kb;
    int j0;
    float db;
    argmax(mine, kb, j0, db);
    // every thread has read the counts (the argmax synchronised the team):
    // the waiting records are consumed
    if (tt == 0 && (in_l | in_r)) {
        bn[(size_t)sid * 2 + 0] = 0u;
        bn[(size_t)sid * 2 + 1] = 0u;
    }

    int n = 0;
    uint32_t n_l = 0, n_r = 0;  // records sent to the left and right neighbours
    bool conv = false, touch_l = false, touch_r = false;
    BoundaryRec* __restrict__ box_l =
        sd.left >= 0 ? a.box + ((size_t)sd.left * 2 + 1) * a.box_cap : nullptr;
    BoundaryRec* __restrict__ box_r =
        sd.right >= 0 ? a.box + ((size_t)sd.right * 2 + 0) * a.box_cap : nullptr;

    // at most kWaveRecs updates per run (the launcher checks the cap)
    for (;;) {
        // per iteration, so that the per-atom constants are read from LDS where
        // they are used instead of being held in registers across the loop
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        if (key_value(kb) < eps_stop) {
            conv = true;
            break;
        }
        if (n == a.cap)
            break;
        const int k0 = 31 - (int)(kb & 31u);
        if (k0 >= K) {  // a padded atom wins only when every candidate is 0
            conv = true;
            break;
        }
        const float delta = db;
        const int wlo = j0 - (W - 1) > 0 ? j0 - (W - 1) : 0;
        const int whi = j0 + (W - 1) < Lm - 1 ? j0 + (W - 1) : Lm - 1;
        tlo = wlo < tlo ? wlo : tlo;
        thi = whi > thi ? whi : thi;

        if (tt == j0) {
            // owner of the updated coordinate: new Z (exactly 0 when the soft
            // threshold is active), in registers and in the double Z in HBM
            float* up = reinterpret_cast<float*>(u + (k0 / 4) * NT) + (k0 % 4);
            const float zo = *up;
            const bool zr = fabsf(fmaf(cn2[k0 / 4][k0 % 4], zo, pick<0, KP, KQ>(g, k0))) <= lam;
            const float zn = zr ? 0.0f : zo + delta;
            *up = zn;
            zs32[(int64_t)k0 * L + b + j0] = zn;
            double* zp = Zs + (int64_t)k0 * L + b + j0;
            if (zr)
                *zp = 0.0;
            else
                unsafeAtomicAdd(zp, (double)delta);  // single owner: deterministic
            if (a.trace) {
                const unsigned long long r = atomicAdd(&a.counters->trace_n, 1ull);
                if ((long long)r < a.trace_cap) {
                    dicod_trace_rec rec;
                    rec.phase = a.phase;
                    rec.seg = sid;
                    rec.k0 = k0;
                    rec.n_local = n;
                    rec.t0 = (int64_t)b + j0;
                    rec.delta = (double)delta;
                    a.trace[r] = rec;
                }
            }
        }
        const bool to_l = j0 - (W - 1) < 0 && sd.left >= 0;
        const bool to_r = j0 + (W - 1) >= Lm && sd.right >= 0;
        if ((to_l || to_r) && tt == 0) {
            BoundaryRec rc;
            rc.k0 = k0;
            rc.t0 = b + j0;
            rc.delta = delta;
            rc.seq = 0;
            if (to_l) {
                if (base_l + n_l < (uint32_t)a.box_cap)
                    box_l[base_l + n_l] = rc;
                else
                    atomicAdd(&a.counters->box_overflow, 1ull);
            }
            if (to_r) {
                if (base_r + n_r < (uint32_t)a.box_cap)
                    box_r[base_r + n_r] = rc;
                else
                    atomicAdd(&a.counters->box_overflow, 1ull);
            }
        }
        n_l += to_l ? 1u : 0u;
        n_r += to_r ? 1u : 0u;
        touch_l |= to_l;
        touch_r |= to_r;

        // eq. (3) over the own positions of the window
        const int dj = tt - j0 + (W - 1);
        if (own && dj >= 0 && dj < nd) {
            const f4* srow = reinterpret_cast<const f4*>(St + ((size_t)k0 * nd + dj) * KP);
            f4 sv[KQ];
#pragma unroll
            for (int i = 0; i < KQ; ++i)
                sv[i] = srow[i];
            // all rows in flight before the first use (the scheduler would
            // otherwise trade them for registers and wait for each in turn)
            __builtin_amdgcn_sched_barrier(0);
            axpy_state<KQ, KL>(g, sv, delta);
            mine = best_key<KQ, KL, NT>(g, u, cn2, cinv, lam);
        }
        ++n;
        argmax(mine, kb, j0, db);
    }

    // own g of every position the run changed
    if (own && tt >= tlo && tt <= thi) {
        float* pg = gs + b + tt;
#pragma unroll
        for (int i = 0; i < KQ; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (4 * i + c < K)
                    *pg = g[i][c];
                pg += L;
            }
    }

    if (tt == 0) {
        if (n > 0) {
            atomicAdd(&a.phase_upd[(size_t)sd.sig * a.phase_stride + a.phase],
                      (unsigned long long)n);
            atomicAdd(&a.sig_upd[sd.sig], (unsigned long long)n);
            atomicMax(&a.sig_last_upd[sd.sig], a.phase);
            atomicAdd(&a.counters->seg_runs, 1ull);
            if (a.changed)
                a.changed[sid] = 1u;
        }
        a.dirty[sid] = conv ? 0u : 1u;
        if (touch_l) {
            a.dirty[sd.left] = 1u;
            bn[(size_t)sd.left * 2 + 1] = base_l + n_l < (uint32_t)a.box_cap
                                              ? base_l + n_l : (uint32_t)a.box_cap;
        }
        if (touch_r) {
            a.dirty[sd.right] = 1u;
            bn[(size_t)sd.right * 2 + 0] = base_r + n_r < (uint32_t)a.box_cap
                                               ? base_r + n_r : (uint32_t)a.box_cap;
        }
    }
}

template <int KQ, int KL>
hipError_t launch_kl(const PhaseArgs& a, hipStream_t s)
{
    if (a.lm_max <= 64) {
        hipLaunchKernelGGL((k_lgcd_wave<KQ, KL, 1>), dim3((unsigned)((a.n_list + 3) / 4)),
                           dim3(256), 0, s, a);
    } else if (a.lm_max <= 128) {
        hipLaunchKernelGGL((k_lgcd_wave<KQ, KL, 2>), dim3((unsigned)a.n_list), dim3(128), 0, s,
                           a);
    } else {
        hipLaunchKernelGGL((k_lgcd_wave<KQ, KL, 4>), dim3((unsigned)a.n_list), dim3(256), 0, s,
                           a);
    }
    return hipGetLastError();
}

// KL: real atoms in the last group of four when only that group is padded;
// otherwise the padded atoms are carried as zeros (KL = 4)
template <int KQ>
hipError_t launch_kq(const PhaseArgs& a, hipStream_t s)
{
    switch (wave_last_group(a.K, KQ)) {
    case 1: return launch_kl<KQ, 1>(a, s);
    case 2: return launch_kl<KQ, 2>(a, s);
    case 3: return launch_kl<KQ, 3>(a, s);
    default: return launch_kl<KQ, 4>(a, s);
    }
}

}  // namespace

int lgcd_wave_box_cap() { return kWaveRecs; }

bool lgcd_wave_supported(int K, int lm_max, int cap, bool fp64)
{
    return !fp64 && lgcd_k_padded(K, false) > 0 && lgcd_k_padded(K, false) <= 32 &&
           lm_max >= 1 && lm_max <= 256 && cap >= 1 && cap <= kWaveRecs;
}

hipError_t launch_lgcd_wave(const PhaseArgs& a, hipStream_t s)
{
    if (a.n_list <= 0)
        return hipSuccess;
    if (a.dicod || !lgcd_wave_supported(a.K, a.lm_max, a.cap, false) || !a.box || !a.box_n ||
        !a.z32 || a.box_cap < a.cap || a.box_cap > kWaveRecs)
        return hipErrorInvalidValue;
    switch (lgcd_k_padded(a.K, false) / 4) {
    case 1: return launch_kq<1>(a, s);
    case 2: return launch_kq<2>(a, s);
    case 4: return launch_kq<4>(a, s);
    case 7: return launch_kq<7>(a, s);
    case 8: return launch_kq<8>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dicod
