// Free-running register-state LGCD kernel: Algorithm 2 (Sec. 2.2) without
// phase barriers (gfx950).
//
// Every segment C_m is a worker of Algorithm 2: it applies the boundary
// updates its neighbours sent, then repeatedly picks the coordinate of
// largest |Delta Z| in C_m (eq. (pb_coord)), applies it and the eq. (3)
// update of its own part of the 2W - 1 window, and sends (k0, t0, delta) to a
// neighbour whose positions the window reaches.  Workers run concurrently
// and independently: two adjacent workers may pick coordinates within W of
// each other before either has received the other's message -- the
// interfering updates of Sec. 3 (Prop. A.2), which converge under H1.
//
// Mapping.  A team (1, 2 or 4 waves; the same layout as the coloured
// register-state kernel: thread j owns position j of the segment, its K
// values of g in registers and of Z in an LDS column) is persistent: it
// loops over the segments sid = team, team + n_teams, ... for up to `sweeps`
// passes, running each segment that is dirty or has records waiting, and
// stops after a pass in which none ran.  A run does at most `cap` updates.
//
// Messages.  ring[s][0] holds the records of the left neighbour, ring[s][1]
// those of the right one; each ring has one producer and one consumer.  The
// producer writes a record, then publishes the counter ring_w with release
// order; the consumer reads ring_w with acquire order, copies the records
// into LDS, applies them and publishes ring_r.  A full ring is counted in
// box_overflow (the host then reports a device error); with the capacity of
// lgcd_async_ring_cap it cannot fill.  Nothing waits: a record that arrives
// after its consumer read ring_w is applied in the consumer's next run (next
// pass or next launch), and the host relaunches until a launch applies no
// update.
//
// Trace (a.trace): updates carry their number in selection order (counter
// upd_seq) in n_local; an application of a neighbour's record is logged with
// k0 = -1 - atom, n_local = the record's update number and t0 = upd_seq when
// applied, so the host can tell which pairs of updates were chosen without
// each other's effect.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "dicod_internal.h"
#include "lgcd_wave_util.h"

namespace dicod {
namespace {

constexpr int kStage = 2 * kWaveRecs;  // records staged in LDS per pass

__device__ __forceinline__ uint32_t load_acquire(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_release(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int TW>
__device__ __forceinline__ void team_sync()
{
    if (TW > 1)
        __syncthreads();
    else
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <int KQ, int KL, int TW>
__global__ void __launch_bounds__(TW == 2 ? 128 : 256)
__attribute__((amdgpu_waves_per_eu(KQ == 8 ? (TW == 1 ? 3 : 4) : (TW == 1 ? 4 : 5))))
k_lgcd_async(PhaseArgs a, AsyncArgs x)
{
    constexpr int SPB = TW == 1 ? 4 : 1;      // teams per workgroup
    constexpr int NTT = 64 * TW;              // threads per team
    constexpr int KP = 4 * KQ;
    constexpr int NT = SPB * NTT;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int team = TW == 1 ? wave : 0;
    const int tt = TW == 1 ? lane : (int)threadIdx.x;

    __shared__ f4 s_cst[SPB][2][KQ];
    __shared__ f4 s_u[KQ * NT];
    __shared__ WSlot s_slot[2][TW];
    __shared__ BoundaryRec s_in[SPB][kStage];
    __shared__ uint32_t s_hdr[SPB][8];
    f4* __restrict__ u = s_u + threadIdx.x;

    const int team_id = blockIdx.x * SPB + team;
    if (team_id >= x.n_teams)
        return;  // a whole team (TW = 1: one wave without block barriers)

    const int K = a.K;
    const int W = a.W;
    const int nd = 2 * W - 1;
    const float* __restrict__ St = reinterpret_cast<const float*>(a.S);  // [K][nd][KP]
    f4* cn2 = s_cst[team][0];
    f4* cinv = s_cst[team][1];
    for (int k = tt; k < KP; k += NTT) {
        reinterpret_cast<float*>(cn2)[k] = k < K ? reinterpret_cast<const float*>(a.n2)[k] : 1.0f;
        reinterpret_cast<float*>(cinv)[k] =
            k < K ? reinterpret_cast<const float*>(a.inv_n2)[k] : 1.0f;
    }
    team_sync<TW>();
    uint32_t* __restrict__ hdr = s_hdr[team];
    BoundaryRec* rin = s_in[team];
    int it = 0;  // argmax slot parity (TW > 1), continued across runs

    for (int sweep = 0; sweep < x.sweeps; ++sweep) {
        bool ran = false;
        for (int sid = team_id; sid < a.n_seg; sid += x.n_teams) {
            const SegDesc sd = a.segs[sid];
            // the segment's header, read once for the team: own work, records
            // waiting on each side, and where this run's records to each
            // neighbour start (this segment is their only producer)
            team_sync<TW>();  // the previous run's reads of hdr and s_in are done
            if (tt == 0) {
                hdr[0] = a.dirty[sid];
                hdr[1] = load_acquire(x.ring_w + (size_t)sid * 2 + 0);
                hdr[2] = load_acquire(x.ring_w + (size_t)sid * 2 + 1);
                hdr[3] = x.ring_r[(size_t)sid * 2 + 0];
                hdr[4] = x.ring_r[(size_t)sid * 2 + 1];
                hdr[5] = sd.left >= 0 ? x.ring_w[(size_t)sd.left * 2 + 1] : 0u;
                hdr[6] = sd.right >= 0 ? x.ring_w[(size_t)sd.right * 2 + 0] : 0u;
                // consumer positions of the outgoing rings: they only grow, so
                // the space computed from them is a lower bound
                const uint32_t rl = sd.left >= 0 ? load_acquire(x.ring_r + (size_t)sd.left * 2 + 1)
                                                 : 0u;
                const uint32_t rr = sd.right >= 0
                                        ? load_acquire(x.ring_r + (size_t)sd.right * 2 + 0) : 0u;
                const uint32_t fl = (uint32_t)x.ring_cap - (hdr[5] - rl);
                const uint32_t fr = (uint32_t)x.ring_cap - (hdr[6] - rr);
                hdr[7] = fl < fr ? fl : fr;
            }
            team_sync<TW>();
            const uint32_t dirty = __builtin_amdgcn_readfirstlane(hdr[0]);
            const uint32_t w_l = __builtin_amdgcn_readfirstlane(hdr[1]);
            const uint32_t w_r = __builtin_amdgcn_readfirstlane(hdr[2]);
            const uint32_t r_l = __builtin_amdgcn_readfirstlane(hdr[3]);
            const uint32_t r_r = __builtin_amdgcn_readfirstlane(hdr[4]);
            const uint32_t base_l = __builtin_amdgcn_readfirstlane(hdr[5]);
            const uint32_t base_r = __builtin_amdgcn_readfirstlane(hdr[6]);
            const uint32_t room = __builtin_amdgcn_readfirstlane(hdr[7]);
            const uint32_t n_wl = w_l - r_l, n_wr = w_r - r_r;
            if (dirty == 0u && n_wl == 0u && n_wr == 0u)
                continue;
            ran = true;

            const int b = sd.b;
            const int Lm = sd.e - sd.b;
            const int64_t L = sd.L;
            float* __restrict__ gs = reinterpret_cast<float*>(a.g) + sd.z_off;
            double* __restrict__ Zs = a.Z + sd.z_off;
            float* __restrict__ zs32 = a.z32 + sd.z_off;
            const float lam = (float)a.sigs[sd.sig].lam;
            const float eps_stop = (float)a.sigs[sd.sig].eps_stop;

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
                        if (4 * i + c + 1 < K) {
                            pg += L;
                            pz += L;
                        }
                    }
            }
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
            int tlo = INT_MAX, thi = -1;

            // the neighbours' records: left ring first, then the right one,
            // each in the order written, through LDS in passes of kStage
            const int n_in = (int)(n_wl + n_wr);
            if (n_in > 0)  // every thread reads records published to thread 0's acquire
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            for (int c0 = 0; c0 < n_in; c0 += kStage) {
                const int cn = n_in - c0 < kStage ? n_in - c0 : kStage;
                for (int i = tt; i < cn; i += NTT) {
                    const int q = c0 + i;
                    const int side = q < (int)n_wl ? 0 : 1;
                    const uint32_t idx = side == 0 ? r_l + (uint32_t)q
                                                   : r_r + (uint32_t)(q - (int)n_wl);
                    rin[i] = x.ring[((size_t)sid * 2 + side) * x.ring_cap +
                                    idx % (uint32_t)x.ring_cap];
                }
                team_sync<TW>();
                if (a.trace && tt == 0) {
                    const unsigned long long now = __hip_atomic_load(
                        &a.counters->upd_seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    for (int i = 0; i < cn; ++i) {
                        const unsigned long long r = atomicAdd(&a.counters->trace_n, 1ull);
                        if ((long long)r < a.trace_cap) {
                            dicod_trace_rec rec;
                            rec.phase = a.phase;
                            rec.seg = sid;
                            rec.k0 = -1 - rin[i].k0;
                            rec.n_local = rin[i].seq;
                            rec.t0 = (int64_t)now;
                            rec.delta = (double)rin[i].delta;
                            a.trace[r] = rec;
                        }
                    }
                }
                for (int r = 0; r < cn; ++r) {
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
                team_sync<TW>();  // the staged records are consumed
            }
            // the records are applied: their slots are free for the producers
            if (tt == 0 && n_in > 0) {
                if (n_wl)
                    store_release(x.ring_r + (size_t)sid * 2 + 0, w_l);
                if (n_wr)
                    store_release(x.ring_r + (size_t)sid * 2 + 1, w_r);
            }

            auto argmax = [&](unsigned mine, unsigned& kb, int& j0, float& db)
                __attribute__((always_inline)) {
                const unsigned wk = wave_max_u32(mine);
                const int wl = first_lane(mine == wk);
                const int k0w = 31 - (int)(wk & 31u);
                const int kk = k0w < KP ? k0w : 0;
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

            int n = 0;
            uint32_t n_l = 0, n_r = 0;
            bool conv = false;
            BoundaryRec* __restrict__ ring_l =
                sd.left >= 0 ? x.ring + ((size_t)sd.left * 2 + 1) * x.ring_cap : nullptr;
            BoundaryRec* __restrict__ ring_r =
                sd.right >= 0 ? x.ring + ((size_t)sd.right * 2 + 0) * x.ring_cap : nullptr;
            for (;;) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                if (key_value(kb) < eps_stop) {
                    conv = true;
                    break;
                }
                if (n == a.cap)
                    break;
                const int k0 = 31 - (int)(kb & 31u);
                if (k0 >= K) {
                    conv = true;
                    break;
                }
                const float delta = db;
                const int wlo = j0 - (W - 1) > 0 ? j0 - (W - 1) : 0;
                const int whi = j0 + (W - 1) < Lm - 1 ? j0 + (W - 1) : Lm - 1;
                tlo = wlo < tlo ? wlo : tlo;
                thi = whi > thi ? whi : thi;

                if (tt == j0) {
                    float* up = reinterpret_cast<float*>(u + (k0 / 4) * NT) + (k0 % 4);
                    const float zo = *up;
                    const bool zr =
                        fabsf(fmaf(cn2[k0 / 4][k0 % 4], zo, pick<0, KP, KQ>(g, k0))) <= lam;
                    const float zn = zr ? 0.0f : zo + delta;
                    *up = zn;
                    zs32[(int64_t)k0 * L + b + j0] = zn;
                    double* zp = Zs + (int64_t)k0 * L + b + j0;
                    if (zr)
                        *zp = 0.0;
                    else
                        unsafeAtomicAdd(zp, (double)delta);  // single owner: deterministic
                }
                const bool to_l = j0 - (W - 1) < 0 && sd.left >= 0;
                const bool to_r = j0 + (W - 1) >= Lm && sd.right >= 0;
                if (tt == 0) {
                    int seq = 0;
                    if (a.trace) {
                        seq = (int)atomicAdd(&a.counters->upd_seq, 1ull);
                        const unsigned long long r = atomicAdd(&a.counters->trace_n, 1ull);
                        if ((long long)r < a.trace_cap) {
                            dicod_trace_rec rec;
                            rec.phase = a.phase;
                            rec.seg = sid;
                            rec.k0 = k0;
                            rec.n_local = seq;
                            rec.t0 = (int64_t)b + j0;
                            rec.delta = (double)delta;
                            a.trace[r] = rec;
                        }
                    }
                    BoundaryRec rc;
                    rc.k0 = k0;
                    rc.t0 = b + j0;
                    rc.delta = delta;
                    rc.seq = seq;
                    // the record is written before its counter is published
                    // (release order), so a consumer that sees the counter
                    // sees the record
                    if (to_l) {
                        if (n_l < room) {
                            ring_l[(base_l + n_l) % (uint32_t)x.ring_cap] = rc;
                            store_release(x.ring_w + (size_t)sd.left * 2 + 1, base_l + n_l + 1u);
                        } else {
                            atomicAdd(&a.counters->box_overflow, 1ull);
                        }
                    }
                    if (to_r) {
                        if (n_r < room) {
                            ring_r[(base_r + n_r) % (uint32_t)x.ring_cap] = rc;
                            store_release(x.ring_w + (size_t)sd.right * 2 + 0, base_r + n_r + 1u);
                        } else {
                            atomicAdd(&a.counters->box_overflow, 1ull);
                        }
                    }
                }
                n_l += to_l ? 1u : 0u;
                n_r += to_r ? 1u : 0u;

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
            }
        }
        if (!ran)
            break;
    }
}

template <int KQ, int KL, int TW>
int teams_of(int n_seg, int n_cu)
{
    constexpr int SPB = TW == 1 ? 4 : 1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_lgcd_async<KQ, KL, TW>,
                                                     TW == 2 ? 128 : 256, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    const long long cap = (long long)nb * n_cu * SPB;
    return (int)(n_seg < cap ? n_seg : cap);
}

template <int KQ, int KL>
int teams_kl(int lm_max, int n_seg, int n_cu)
{
    if (lm_max <= 64)
        return teams_of<KQ, KL, 1>(n_seg, n_cu);
    if (lm_max <= 128)
        return teams_of<KQ, KL, 2>(n_seg, n_cu);
    return teams_of<KQ, KL, 4>(n_seg, n_cu);
}

template <int KQ>
int teams_kq(int K, int lm_max, int n_seg, int n_cu)
{
    switch (wave_last_group(K, KQ)) {
    case 1: return teams_kl<KQ, 1>(lm_max, n_seg, n_cu);
    case 2: return teams_kl<KQ, 2>(lm_max, n_seg, n_cu);
    case 3: return teams_kl<KQ, 3>(lm_max, n_seg, n_cu);
    default: return teams_kl<KQ, 4>(lm_max, n_seg, n_cu);
    }
}

template <int KQ, int KL>
hipError_t launch_kl(const PhaseArgs& a, const AsyncArgs& x, hipStream_t s)
{
    if (a.lm_max <= 64) {
        hipLaunchKernelGGL((k_lgcd_async<KQ, KL, 1>), dim3((unsigned)((x.n_teams + 3) / 4)),
                           dim3(256), 0, s, a, x);
    } else if (a.lm_max <= 128) {
        hipLaunchKernelGGL((k_lgcd_async<KQ, KL, 2>), dim3((unsigned)x.n_teams), dim3(128), 0,
                           s, a, x);
    } else {
        hipLaunchKernelGGL((k_lgcd_async<KQ, KL, 4>), dim3((unsigned)x.n_teams), dim3(256), 0,
                           s, a, x);
    }
    return hipGetLastError();
}

template <int KQ>
hipError_t launch_kq(const PhaseArgs& a, const AsyncArgs& x, hipStream_t s)
{
    switch (wave_last_group(a.K, KQ)) {
    case 1: return launch_kl<KQ, 1>(a, x, s);
    case 2: return launch_kl<KQ, 2>(a, x, s);
    case 3: return launch_kl<KQ, 3>(a, x, s);
    default: return launch_kl<KQ, 4>(a, x, s);
    }
}

}  // namespace

int lgcd_async_ring_cap(int cap, int sweeps) { return 2 * cap * sweeps; }

int lgcd_async_teams(int K, int lm_max, int n_seg, int n_cu)
{
    switch (lgcd_k_padded(K, false) / 4) {
    case 1: return teams_kq<1>(K, lm_max, n_seg, n_cu);
    case 2: return teams_kq<2>(K, lm_max, n_seg, n_cu);
    case 4: return teams_kq<4>(K, lm_max, n_seg, n_cu);
    case 7: return teams_kq<7>(K, lm_max, n_seg, n_cu);
    case 8: return teams_kq<8>(K, lm_max, n_seg, n_cu);
    default: return 0;
    }
}

hipError_t launch_lgcd_async(const PhaseArgs& a, const AsyncArgs& x, hipStream_t s)
{
    if (a.n_seg <= 0)
        return hipSuccess;
    if (a.dicod || !lgcd_wave_supported(a.K, a.lm_max, a.cap, false) || !a.z32 || !x.ring ||
        !x.ring_w || !x.ring_r || x.n_teams < 1 || x.sweeps < 1 ||
        x.ring_cap < lgcd_async_ring_cap(a.cap, x.sweeps))
        return hipErrorInvalidValue;
    switch (lgcd_k_padded(a.K, false) / 4) {
    case 1: return launch_kq<1>(a, x, s);
    case 2: return launch_kq<2>(a, x, s);
    case 4: return launch_kq<4>(a, x, s);
    case 7: return launch_kq<7>(a, x, s);
    case 8: return launch_kq<8>(a, x, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dicod
