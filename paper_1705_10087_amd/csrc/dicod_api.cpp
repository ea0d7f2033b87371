// Host runtime and C ABI (include/dicod.h) of the gfx950 LGCD library.
//
// Each solve follows Algorithm 3 of Moreau, Oudre & Vayatis (ICML 2018) over
// M time segments (Sec. 2.2):
//   1. beta at Z = 0 (Algorithm 1 init) on MFMA, in double;
//   2. lambda = |lambda| * max |beta| when lambda is relative;
//   3. coloured phases of segment runs (kernels.hip: k_lgcd_phase, or
//      k_lgcd_phase_gm when the state stays in HBM) until C consecutive
//      phases apply no update;
//   4. a double-precision check of max |Delta Z| over all coordinates (the
//      stop test of Sec. 2.1); in the FP32 policy a failed check refreshes g
//      from the double recompute and resumes step 3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <vector>

#include "dicod_internal.h"
#include "dicod_serve.h"

using namespace dicod;

namespace {

thread_local std::string g_init_error;

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    bool owned = true;  // false: a view into the static scratch (never freed)
    ~DevBuf() { release(); }
    void release()
    {
        if (p && owned)
            (void)hipFree(p);
        p = nullptr;
        n = 0;
        owned = true;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// The allocation-free solve (dicod_solve_device_noalloc) sets t_arena: every
// workspace buffer is then carved, 256-byte aligned, from the static device
// scratch instead of being allocated; a request beyond its size fails and
// records how much the problem needs.
struct Arena {
    unsigned char* base = nullptr;
    size_t cap = 0, off = 0, need = 0;
    bool overflow = false;
};
thread_local Arena* t_arena = nullptr;

hipError_t ensure(DevBuf& b, size_t bytes)
{
    if (bytes == 0)
        bytes = 16;
    if (t_arena) {
        if (!b.owned && b.p && b.n >= bytes)
            return hipSuccess;  // carved earlier in this call
        const size_t off = (t_arena->off + 255) & ~(size_t)255;
        if (off + bytes > t_arena->cap) {
            t_arena->overflow = true;
            t_arena->need = std::max(t_arena->need, off + bytes);
            return hipErrorOutOfMemory;
        }
        b.release();
        b.p = t_arena->base + off;
        b.n = bytes;
        b.owned = false;
        t_arena->off = off + bytes;
        return hipSuccess;
    }
    if (b.n >= bytes)
        return hipSuccess;
    b.release();
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess)
        b.n = bytes;
    else
        b.p = nullptr;
    return e;
}

struct Workspace {
    DevBuf X, Zout;                       // staging for the host-pointer API
    DevBuf beta0, g, g64;                 // [K][L] per signal (g64: double finish)
    DevBuf sig, segs, lists[kMaxColors];
    DevBuf tilesL, tilesC, tilesA, tilesN;
    DevBuf nzmask;                        // non-zero masks of Z for the check kernels
    DevBuf dirty, phase_upd, sig_upd, sig_last, counters;
    DevBuf part, results, lmax, done, thr, ebits;
    DevBuf msg, msg_n;                    // DICOD schedule: boundary messages
    DevBuf box, box_n, z32;               // register kernel: mailboxes, float copy of Z
    DevBuf ring, ring_wr;                 // free-running schedule: rings and their counters
    DevBuf changed;                       // per segment: Z changed since the last check
    DevBuf trace;
    DevBuf slots, lamin;                  // device-side lambda: signal indices, inputs
    // host copies of what the read-only plan tables hold on the device: an
    // identical plan is not uploaded again
    std::vector<unsigned char> sh_segs, sh_lists[kMaxColors], sh_tL, sh_tC, sh_tA, sh_tN, sh_slots;
};

}  // namespace

struct dicod_ctx {
    dicod_config cfg;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;          // double beta0, overlapped with the descent
    int n_cu = 256;                      // compute units of the device
    hipEvent_t ev_in = nullptr, ev_beta = nullptr;
    std::string err;
    // resident dictionary
    bool has_dict = false;
    int K = 0, P = 0, W = 0;
    double dnorm_max = 0.0;              // max_k |D_k|_2 (error bound of the bf16 split)
    DevBuf D64, D32, S64, S32, n2_64, inv64, n2_32, inv32;
    DevBuf St32, St64;  // phase-kernel layouts of S (float, double)
    DevBuf Sc64;        // S with rows padded to 2W doubles, for the double check
    DevBuf Dsp;         // bf16 hi/lo split of D for the MIXED correlation
    Workspace ws;
    Workspace ws_scratch;                 // views into the static scratch (noalloc solve)
    void* scratch = nullptr;              // device address of the static scratch
    unsigned long long* h_upd = nullptr;  // pinned copy of per-phase counts
    size_t h_upd_cap = 0;
    hipEvent_t ev_poll[2] = {nullptr, nullptr};  // queued chunks of phases
    unsigned char* h_pin = nullptr;       // pinned staging of per-round uploads
    size_t h_pin_cap = 0;
    std::vector<hipEvent_t> ev_pool;
    int64_t last_trace_n = 0;
    dicod::Server* server = nullptr;
    // autotuner: chosen schedule per length bucket, and the schedule forced on
    // the solves of a tuning trial
    std::map<int, dicod_tune_entry> tuning;
    const dicod_tune_entry* sched_force = nullptr;
};

namespace {

int fail(dicod_ctx* ctx, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_init_error = buf;
    return code;
}

#define HIPCHECK(ctx, expr)                                                          \
    do {                                                                             \
        hipError_t _e = (expr);                                                      \
        if (_e != hipSuccess)                                                        \
            return fail((ctx), _e == hipErrorOutOfMemory ? DICOD_ENOMEM : DICOD_EDEVICE, \
                        "%s: %s", #expr, hipGetErrorString(_e));                     \
    } while (0)

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Offsets in the pinned staging of a solve of n_sig signals: uploads
// (done flags at 0, lambda inputs, descriptors), then read-backs (check
// results, final statistics).
struct PinLayout {
    size_t lam, sig, res, supd, slast, lbits, cnt, need;
};

PinLayout pin_layout(int n_sig)
{
    auto al256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    PinLayout l;
    l.lam = al256((size_t)n_sig * sizeof(uint32_t));
    l.sig = l.lam + al256((size_t)n_sig * sizeof(double));
    l.res = l.sig + al256((size_t)n_sig * sizeof(SigDesc));
    l.supd = l.res + al256((size_t)n_sig * sizeof(CheckResult));
    l.slast = l.supd + al256((size_t)n_sig * sizeof(unsigned long long));
    l.lbits = l.slast + al256((size_t)n_sig * sizeof(int));
    l.cnt = l.lbits + al256((size_t)n_sig * sizeof(unsigned long long));
    l.need = l.cnt + sizeof(Counters);
    return l;
}

size_t pinned_bytes(int n_sig) { return pin_layout(n_sig).need; }

hipEvent_t pool_event(dicod_ctx* ctx, size_t i);

double elapsed_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess)
        return 0.0;
    return (double)ms;
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Shortest segment for C colours: an update changes beta on the W - 1
// positions on each side of it (eq. (3)), so a window may only reach the
// adjacent segments when every segment is at least W - 1 long; segments of one
// colour run together and must stay 2W - 2 apart (two half-windows).
int64_t min_segment(int W, int C)
{
    const int64_t reach = W > 1 ? (int64_t)W - 1 : 1;
    if (C <= 1)  // Algorithm 2: a window may only reach the adjacent segments
        return reach;
    const int64_t gap = (2 * (int64_t)W - 2 + (C - 2)) / (C - 1);
    return std::max<int64_t>(reach, gap);
}

// Segment count M chosen by the library: the largest M allowed by
// min_segment (with 2 colours this is close to the paper's optimum
// M* ~ T / (2W) of Corollary 1; 3 colours give segments of W - 1 or W
// coefficients, about the paper's M = T / W choice for SeqDICOD).
int auto_segments(int64_t L, int W, int C)
{
    const int64_t M = L / min_segment(W, C);
    return M < 1 ? 1 : (int)std::min<int64_t>(M, INT32_MAX);
}

// Length bucket of the tuning table: floor(log2(L)).
int length_bucket(int64_t L)
{
    int b = 0;
    while (L > 1) {
        L >>= 1;
        ++b;
    }
    return b;
}

// Segment count for a longest segment of seg_len positions: ceil(L / seg_len),
// lowered to the largest count that keeps every segment at least
// min_segment(W, C) long.
int tuned_segments(int64_t L, int W, int C, int seg_len)
{
    int64_t M = (L + seg_len - 1) / std::max(seg_len, 1);
    M = std::max<int64_t>(1, std::min<int64_t>(M, L));
    if (M > 1 && L / M < min_segment(W, C))
        M = auto_segments(L, W, C);
    return (int)std::min<int64_t>(M, INT32_MAX);
}

bool find_tuning(const dicod_ctx* ctx, int bucket, dicod_tune_entry* e);

}  // namespace

// ---------------------------------------------------------------------------
// config, init, finalize, errors
// ---------------------------------------------------------------------------
extern "C" int dicod_config_init(dicod_config* cfg)
{
    if (!cfg)
        return DICOD_EINVAL;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->device = 0;
    cfg->precision = DICOD_PREC_FP32;
    cfg->schedule = DICOD_SCHED_EVENODD;
    cfg->update_cap = -1;
    cfg->max_phases = 1000000;
    cfg->max_refresh = 8;
    cfg->phases_per_poll = 16;
    cfg->inner_eps_factor = 0.5;
    cfg->hbm_budget_bytes = 0;
    cfg->max_inflight = 64;
    cfg->timing = 0;
    cfg->trace_capacity = 0;
    cfg->state_in_lds = 1;
    cfg->fp64_polish_after = 1;
    cfg->colors = 3;
    cfg->verify_from_scratch = 0;
    cfg->reg_state = 1;
    cfg->autotune = 0;
    cfg->screen = 0;
    return DICOD_OK;
}

extern "C" int dicod_init(dicod_ctx** out, const dicod_config* cfg)
{
    if (!out)
        return fail(nullptr, DICOD_EINVAL, "dicod_init: out is NULL");
    *out = nullptr;
    dicod_config c;
    if (cfg)
        c = *cfg;
    else
        dicod_config_init(&c);
    if (c.precision < DICOD_PREC_FP64 || c.precision > DICOD_PREC_MIXED)
        return fail(nullptr, DICOD_EINVAL, "dicod_init: unknown precision %d", c.precision);
    if (c.schedule != DICOD_SCHED_EVENODD && c.schedule != DICOD_SCHED_DICOD &&
        c.schedule != DICOD_SCHED_ASYNC)
        return fail(nullptr, DICOD_EINVAL, "dicod_init: unknown schedule %d", c.schedule);
    if (c.schedule == DICOD_SCHED_DICOD && c.update_cap != -1 &&
        (c.update_cap < 1 || c.update_cap > 1024))
        return fail(nullptr, DICOD_EINVAL,
                    "dicod_init: the DICOD schedule needs update_cap in 1..1024 or -1");
    if (c.update_cap < -1 || c.max_phases < 2 || c.max_refresh < 0 ||
        c.phases_per_poll < 1 || !(c.inner_eps_factor > 0.0 && c.inner_eps_factor <= 1.0) ||
        c.trace_capacity < 0 || c.max_inflight < 1 || c.fp64_polish_after < 0 ||
        c.colors < 2 || c.colors > kMaxColors || c.autotune < 0 || c.autotune > 1 ||
        c.screen < 0 || c.screen > 1)
        return fail(nullptr, DICOD_EINVAL, "dicod_init: invalid configuration field");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(nullptr, DICOD_EDEVICE, "dicod_init: no HIP device visible");
    if (c.device < 0 || c.device >= ndev)
        return fail(nullptr, DICOD_EINVAL, "dicod_init: device %d out of range (%d devices)",
                    c.device, ndev);
    if (hipSetDevice(c.device) != hipSuccess)
        return fail(nullptr, DICOD_EDEVICE, "dicod_init: hipSetDevice(%d) failed", c.device);
    dicod_ctx* ctx = new (std::nothrow) dicod_ctx();
    if (!ctx)
        return fail(nullptr, DICOD_ENOMEM, "dicod_init: out of host memory");
    ctx->cfg = c;
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_beta, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_poll[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_poll[1], hipEventDisableTiming) != hipSuccess) {
        dicod_finalize(ctx);
        return fail(nullptr, DICOD_EDEVICE, "dicod_init: stream or event creation failed");
    }
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c.device) ==
            hipSuccess && n_cu > 0)
        ctx->n_cu = n_cu;
    // set-up of the allocation-free solve: the static scratch's address on this
    // device, pinned staging for one signal and the phase counts, and the
    // events of one solve
    if (dicod::scratch_address(c.device, &ctx->scratch) != hipSuccess || !ctx->scratch) {
        dicod_finalize(ctx);
        return fail(nullptr, DICOD_EDEVICE, "dicod_init: no address for the static scratch");
    }
    const size_t n_upd = (size_t)std::min<int64_t>(c.max_phases, (int64_t)1 << 22) + 1;
    if (hipHostMalloc((void**)&ctx->h_upd, n_upd * sizeof(unsigned long long),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_pin, pinned_bytes(1), hipHostMallocDefault) != hipSuccess) {
        dicod_finalize(ctx);
        return fail(nullptr, DICOD_ENOMEM, "dicod_init: pinned staging");
    }
    ctx->h_upd_cap = n_upd;
    ctx->h_pin_cap = pinned_bytes(1);
    for (size_t i = 0; i < 4; ++i)
        if (!pool_event(ctx, i)) {
            dicod_finalize(ctx);
            return fail(nullptr, DICOD_EDEVICE, "dicod_init: event creation failed");
        }
    *out = ctx;
    return DICOD_OK;
}

extern "C" void dicod_finalize(dicod_ctx* ctx)
{
    if (!ctx)
        return;
    (void)hipSetDevice(ctx->cfg.device);
    if (ctx->server) {
        dicod::server_destroy(ctx->server);
        ctx->server = nullptr;
    }
    if (ctx->stream)
        (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side)
        (void)hipStreamSynchronize(ctx->side);
    for (hipEvent_t e : ctx->ev_pool)
        (void)hipEventDestroy(e);
    if (ctx->ev_in)
        (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_beta)
        (void)hipEventDestroy(ctx->ev_beta);
    for (hipEvent_t e : ctx->ev_poll)
        if (e)
            (void)hipEventDestroy(e);
    if (ctx->h_upd)
        (void)hipHostFree(ctx->h_upd);
    if (ctx->h_pin)
        (void)hipHostFree(ctx->h_pin);
    if (ctx->stream)
        (void)hipStreamDestroy(ctx->stream);
    if (ctx->side)
        (void)hipStreamDestroy(ctx->side);
    delete ctx;
}

extern "C" const char* dicod_last_error(const dicod_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

// ---------------------------------------------------------------------------
// dictionary
// ---------------------------------------------------------------------------
extern "C" int dicod_set_dictionary(dicod_ctx* ctx, const float* D, int K, int P, int W)
{
    if (!ctx)
        return DICOD_EINVAL;
    ctx->err.clear();
    if (!D)
        return fail(ctx, DICOD_EINVAL, "dicod_set_dictionary: D is NULL");
    if (K <= 0 || P <= 0 || W <= 0)
        return fail(ctx, DICOD_EINVAL, "dicod_set_dictionary: K=%d P=%d W=%d must be > 0",
                    K, P, W);
    if (ctx->server) {
        // the serving lanes hold the dictionary's device tables and sizes for
        // the life of the context
        const int64_t open = dicod::server_open_requests(ctx->server);
        return fail(ctx, DICOD_EINVAL,
                    "dicod_set_dictionary: serving active on this context (%lld requests "
                    "not yet polled); the dictionary is fixed until dicod_finalize",
                    (long long)open);
    }
    if (P > kMaxP)
        return fail(ctx, DICOD_ENOTSUP, "dicod_set_dictionary: P=%d > %d channels", P, kMaxP);
    if ((int64_t)K * P * W > (int64_t)1 << 28)
        return fail(ctx, DICOD_ENOTSUP, "dicod_set_dictionary: dictionary too large");
    const size_t n = (size_t)K * P * W;
    std::vector<double> d64(n);
    for (size_t i = 0; i < n; ++i) {
        if (!std::isfinite(D[i]))
            return fail(ctx, DICOD_EINVAL, "dicod_set_dictionary: D[%zu] is not finite", i);
        d64[i] = (double)D[i];
    }
    double dnorm_max = 0.0;
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (size_t i = 0; i < (size_t)P * W; ++i)
            s += d64[(size_t)k * P * W + i] * d64[(size_t)k * P * W + i];
        if (!(s > 0.0))
            return fail(ctx, DICOD_EINVAL, "dicod_set_dictionary: atom %d has zero norm", k);
        dnorm_max = std::max(dnorm_max, std::sqrt(s));
    }
    HIPCHECK(ctx, hipSetDevice(ctx->cfg.device));
    hipStream_t s = ctx->stream;
    const int nd = 2 * W - 1;
    const int Tp = 3 * W - 2;  // padded atom: W - 1 zeros, the atom, W - 1 zeros
    std::vector<double> pad((size_t)K * P * Tp, 0.0);
    for (int k = 0; k < K; ++k)
        for (int p = 0; p < P; ++p)
            for (int t = 0; t < W; ++t)
                pad[((size_t)k * P + p) * Tp + (W - 1) + t] = d64[((size_t)k * P + p) * W + t];
    std::vector<SigDesc> sd(K);
    std::vector<int64_t> pref(K + 1, 0);
    for (int k = 0; k < K; ++k) {
        sd[k].x_off = (int64_t)k * P * Tp;
        sd[k].z_off = (int64_t)k * K * nd;
        sd[k].T = Tp;
        sd[k].L = nd;
        sd[k].seg_base = 0;
        sd[k].M = 1;
        sd[k].lam = 0.0;
        sd[k].eps_stop = 0.0;
        pref[k + 1] = pref[k] + ceil_div(nd, kTile);
    }
    DevBuf dpad, dsig, dpref;
    HIPCHECK(ctx, ensure(ctx->D64, n * sizeof(double)));
    HIPCHECK(ctx, ensure(ctx->D32, n * sizeof(float)));
    HIPCHECK(ctx, ensure(ctx->S64, (size_t)K * K * nd * sizeof(double)));
    HIPCHECK(ctx, ensure(ctx->S32, (size_t)K * K * nd * sizeof(float)));
    HIPCHECK(ctx, ensure(ctx->n2_64, K * sizeof(double)));
    HIPCHECK(ctx, ensure(ctx->inv64, K * sizeof(double)));
    HIPCHECK(ctx, ensure(ctx->n2_32, K * sizeof(float)));
    HIPCHECK(ctx, ensure(ctx->inv32, K * sizeof(float)));
    HIPCHECK(ctx, ensure(dpad, pad.size() * sizeof(double)));
    HIPCHECK(ctx, ensure(dsig, sd.size() * sizeof(SigDesc)));
    HIPCHECK(ctx, ensure(dpref, pref.size() * sizeof(int64_t)));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->D64.p, d64.data(), n * sizeof(double),
                                 hipMemcpyHostToDevice, s));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->D32.p, D, n * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHECK(ctx, hipMemcpyAsync(dpad.p, pad.data(), pad.size() * sizeof(double),
                                 hipMemcpyHostToDevice, s));
    HIPCHECK(ctx, hipMemcpyAsync(dsig.p, sd.data(), sd.size() * sizeof(SigDesc),
                                 hipMemcpyHostToDevice, s));
    HIPCHECK(ctx, hipMemcpyAsync(dpref.p, pref.data(), pref.size() * sizeof(int64_t),
                                 hipMemcpyHostToDevice, s));
    // S_{k,l}[d] as the correlation of every atom with every zero-padded atom.
    HIPCHECK(ctx, launch_corr_f64_x64(ctx->D64.as<double>(), K, P, W, dpad.as<double>(),
                                      dsig.as<SigDesc>(), dpref.as<int64_t>(), K,
                                      pref[K], ctx->S64.as<double>(), s));
    HIPCHECK(ctx, launch_dict_finish(ctx->S64.as<double>(), K, W, ctx->S32.as<float>(),
                                     ctx->n2_64.as<double>(), ctx->inv64.as<double>(),
                                     ctx->n2_32.as<float>(), ctx->inv32.as<float>(), s));
    for (int f64 = 0; f64 < 2; ++f64) {
        const int KP = lgcd_k_padded(K, f64 != 0);
        DevBuf& St = f64 ? ctx->St64 : ctx->St32;
        if (KP < 0) {
            St.release();  // no stale table of a previous dictionary
            continue;      // the phase kernel reports ENOTSUP for this K
        }
        HIPCHECK(ctx, ensure(St, (size_t)K * nd * KP * (f64 ? sizeof(double) : sizeof(float))));
        HIPCHECK(ctx, launch_s_transpose(ctx->S64.as<double>(), K, W, f64 != 0, St.p, s));
    }
    HIPCHECK(ctx, ensure(ctx->Dsp, corr_bf16_dsp_elems(K, P, W) * sizeof(unsigned short)));
    HIPCHECK(ctx, launch_split_d(ctx->D32.as<float>(), K, P, W, ctx->Dsp.as<unsigned short>(), s));
    if (check_kblocks(K, W) > 0) {
        HIPCHECK(ctx, ensure(ctx->Sc64, check_s_elems(K, W) * sizeof(double)));
        HIPCHECK(ctx, hipMemsetAsync(ctx->Sc64.p, 0, check_s_elems(K, W) * sizeof(double), s));
        HIPCHECK(ctx, hipMemcpy2DAsync(ctx->Sc64.p, (size_t)2 * W * sizeof(double), ctx->S64.p,
                                       (size_t)nd * sizeof(double), (size_t)nd * sizeof(double),
                                       (size_t)K * K, hipMemcpyDeviceToDevice, s));
    } else {
        ctx->Sc64.release();  // solves report ENOTSUP for this W
    }
    HIPCHECK(ctx, hipStreamSynchronize(s));
    ctx->K = K;
    ctx->P = P;
    ctx->W = W;
    ctx->dnorm_max = dnorm_max;
    ctx->has_dict = true;
    return DICOD_OK;
}

extern "C" int dicod_get_s_table(dicod_ctx* ctx, double* S_out, double* norms_out)
{
    if (!ctx)
        return DICOD_EINVAL;
    if (!ctx->has_dict)
        return fail(ctx, DICOD_EINVAL, "dicod_get_s_table: no resident dictionary");
    HIPCHECK(ctx, hipSetDevice(ctx->cfg.device));
    const size_t nS = (size_t)ctx->K * ctx->K * (2 * ctx->W - 1);
    if (S_out)
        HIPCHECK(ctx, hipMemcpy(S_out, ctx->S64.p, nS * sizeof(double), hipMemcpyDeviceToHost));
    if (norms_out)
        HIPCHECK(ctx, hipMemcpy(norms_out, ctx->n2_64.p, ctx->K * sizeof(double),
                                hipMemcpyDeviceToHost));
    return DICOD_OK;
}

extern "C" int dicod_check_h1(dicod_ctx* ctx, double* ratio, int* holds)
{
    if (!ctx || !ratio)
        return DICOD_EINVAL;
    ctx->err.clear();
    if (!ctx->has_dict)
        return fail(ctx, DICOD_EINVAL, "dicod_check_h1: no resident dictionary");
    const int K = ctx->K, W = ctx->W, nd = 2 * W - 1;
    std::vector<double> S((size_t)K * K * nd), n2(K);
    const int rc = dicod_get_s_table(ctx, S.data(), n2.data());
    if (rc != DICOD_OK)
        return rc;
    // S[l][k][d + W - 1] = S_{k,l}[d]; every (k, l) pair and shift d != 0
    double worst = 0.0;
    for (int l = 0; l < K; ++l)
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < nd; ++j) {
                if (j == W - 1)
                    continue;
                const double r = std::fabs(S[((size_t)l * K + k) * nd + j]) /
                                 std::sqrt(n2[k] * n2[l]);
                worst = std::max(worst, r);
            }
    *ratio = worst;
    if (holds)
        *holds = worst < 1.0 ? 1 : 0;
    return DICOD_OK;
}

// ---------------------------------------------------------------------------
// the solver
// ---------------------------------------------------------------------------
namespace {

struct Plan {
    std::vector<SigDesc> sig;
    std::vector<SegDesc> segs;
    std::vector<int32_t> list[kMaxColors];
    int colors = 2;   // phase classes; 1 for the DICOD schedule (all segments)
    bool dicod = false;
    // tiles of kTile (L) and of the check (C) positions; mask words (N)
    std::vector<int64_t> prefL, prefC, prefA, prefN;
    int lm_max = 0, lext_max = 0;
    size_t zext = 0;  // extent of the [K][L] arrays (elements)
};

// Where a precision keeps the segment state during a phase: LDS when the
// largest segment fits (and the configuration allows it), else HBM.  Returns
// false when neither kernel can hold the segments.
bool state_fits(const Plan& pl, int K, bool fp64, bool allow_lds, bool* in_lds)
{
    if (allow_lds && pl.lm_max <= 4 * kPhaseThreads &&
        lgcd_lds_bytes(K, pl.lm_max, pl.lext_max, fp64) <= kLdsBytes) {
        *in_lds = true;
        return true;
    }
    *in_lds = false;
    return lgcd_gm_lds_bytes(K, pl.lext_max, fp64) <= kLdsBytes;
}

int make_plan(dicod_ctx* ctx, int colors, int n_sig, const int64_t* T, const int64_t* x_off,
              const double* lam, const int* n_seg, const int64_t* z_off, Plan& pl)
{
    const int K = ctx->K, W = ctx->W;
    const bool fp64 = ctx->cfg.precision == DICOD_PREC_FP64;
    if (check_kblocks(K, W) < 1)
        return fail(ctx, DICOD_ENOTSUP, "W=%d: one row of S does not fit the check kernel", W);
    pl.dicod = ctx->cfg.schedule == DICOD_SCHED_DICOD;
    pl.colors = pl.dicod ? 1 : colors;
    pl.sig.resize(n_sig);
    pl.prefL.assign(n_sig + 1, 0);
    pl.prefC.assign(n_sig + 1, 0);
    pl.prefA.assign(n_sig + 1, 0);
    pl.prefN.assign(n_sig + 1, 0);
    for (int i = 0; i < n_sig; ++i) {
        if (T[i] < W)
            return fail(ctx, DICOD_EINVAL, "signal %d: T=%lld < W=%d", i, (long long)T[i], W);
        if (T[i] > (int64_t)INT32_MAX / 2)
            return fail(ctx, DICOD_ENOTSUP, "signal %d: T=%lld too long", i, (long long)T[i]);
        if (!std::isfinite(lam[i]) || lam[i] == 0.0)
            return fail(ctx, DICOD_EINVAL, "signal %d: lambda must be finite and non-zero", i);
        if (x_off[i] < 0 || z_off[i] < 0)
            return fail(ctx, DICOD_EINVAL, "signal %d: negative offset", i);
        const int64_t L = T[i] - W + 1;
        int M = n_seg ? n_seg[i] : 0;
        if (M < 0)
            return fail(ctx, DICOD_EINVAL, "signal %d: n_seg=%d < 0", i, M);
        if (M == 0)
            M = auto_segments(L, W, pl.colors);
        if (M > L)
            return fail(ctx, DICOD_EINVAL, "signal %d: n_seg=%d > L=%lld", i, M, (long long)L);
        if (M > 1 && L / M < min_segment(W, pl.colors))
            return fail(ctx, DICOD_EINVAL,
                        "signal %d: n_seg=%d gives segments of %lld < %lld coefficients "
                        "(W=%d, %d colours)", i, M, (long long)(L / M),
                        (long long)min_segment(W, pl.colors), W, pl.colors);
        const int64_t lm = ceil_div(L, M);
        int64_t lx = pl.dicod ? lm : lm + 2 * (int64_t)(W - 1);  // DICOD: own positions
        if (lx > L)
            lx = L;
        if (lgcd_gm_lds_bytes(K, (int)lx, fp64) > kLdsBytes)
            return fail(ctx, DICOD_ENOTSUP,
                        "signal %d: segments of %lld coefficients are too long even for the "
                        "HBM-state kernel; use more segments", i, (long long)lm);
        pl.lm_max = std::max(pl.lm_max, (int)lm);
        pl.lext_max = std::max(pl.lext_max, (int)lx);
        SigDesc& s = pl.sig[i];
        s.x_off = x_off[i];
        s.z_off = z_off[i];
        s.T = T[i];
        s.L = L;
        s.seg_base = (int32_t)pl.segs.size();
        s.M = M;
        s.lam = lam[i];
        s.eps_stop = 0.0;
        s.nz_off = pl.prefN[i];
        for (int m = 0; m < M; ++m) {
            SegDesc d;
            d.z_off = z_off[i];
            d.L = (int32_t)L;
            d.b = (int32_t)(((__int128)m * L) / M);
            d.e = (int32_t)(((__int128)(m + 1) * L) / M);
            d.sig = i;
            d.left = m > 0 ? s.seg_base + m - 1 : -1;
            d.right = m < M - 1 ? s.seg_base + m + 1 : -1;
            pl.list[m % pl.colors].push_back(s.seg_base + m);
            pl.segs.push_back(d);
        }
        pl.prefL[i + 1] = pl.prefL[i] + ceil_div(L, kTile);
        pl.prefC[i + 1] = pl.prefC[i] + ceil_div(L, kCheckSpan);
        pl.prefA[i + 1] = pl.prefA[i] + ceil_div((int64_t)K * L, kAbsChunk);
        pl.prefN[i + 1] = pl.prefN[i] + (int64_t)K * ceil_div(L, 64);
        pl.zext = std::max(pl.zext, (size_t)(z_off[i] + (int64_t)K * L));
    }
    return DICOD_OK;
}

template <typename T>
hipError_t upload(DevBuf& b, const std::vector<T>& v, hipStream_t s)
{
    hipError_t e = ensure(b, v.size() * sizeof(T));
    if (e != hipSuccess || v.empty())
        return e;
    return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// Uploads v unless the buffer already holds exactly these bytes (as recorded
// in shadow); for read-only tables.
template <typename T>
hipError_t upload_cached(DevBuf& b, const std::vector<T>& v, std::vector<unsigned char>& shadow,
                         hipStream_t s)
{
    const size_t bytes = v.size() * sizeof(T);
    if (b.p && b.n >= bytes && shadow.size() == bytes &&
        (bytes == 0 || std::memcmp(shadow.data(), v.data(), bytes) == 0))
        return hipSuccess;
    shadow.clear();
    hipError_t e = upload(b, v, s);
    if (e == hipSuccess)
        shadow.assign(reinterpret_cast<const unsigned char*>(v.data()),
                      reinterpret_cast<const unsigned char*>(v.data()) + bytes);
    return e;
}

hipEvent_t pool_event(dicod_ctx* ctx, size_t i)
{
    while (ctx->ev_pool.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[i];
}

}  // namespace

namespace dicod {

// Solves n_sig signals whose X and Z live on the device.  lam_in follows the
// ABI sign convention.  st (optional) receives one entry per signal.
int solve_device_batch(dicod_ctx* ctx, int n_sig, const float* dX, const int64_t* T,
                       const int64_t* x_off, const double* lam_in, double eps,
                       const int* n_seg, double* dZ, const int64_t* z_off,
                       dicod_stats* st, hipStream_t s)
{
    const double t_call0 = now_ms();
    if (!ctx->has_dict)
        return fail(ctx, DICOD_EINVAL, "no resident dictionary (dicod_set_dictionary)");
    if (n_sig <= 0 || !dX || !dZ || !T || !x_off || !lam_in || !z_off)
        return fail(ctx, DICOD_EINVAL, "solve: NULL argument or n_sig <= 0");
    if (!(eps > 0.0) || !std::isfinite(eps))
        return fail(ctx, DICOD_EINVAL, "solve: eps must be finite and > 0");
    const int K = ctx->K, P = ctx->P, W = ctx->W;
    const bool fp64 = ctx->cfg.precision == DICOD_PREC_FP64;
    dicod_config cfg = ctx->cfg;  // colours and cap may come from the tuning table
    Workspace& ws = t_arena ? ctx->ws_scratch : ctx->ws;

    std::vector<int> m_tuned;
    int tuned = 0;
    {
        bool all_auto = true;
        for (int i = 0; n_seg && i < n_sig; ++i)
            all_auto = all_auto && n_seg[i] == 0;
        dicod_tune_entry e;
        bool have = false;
        if (ctx->sched_force) {
            e = *ctx->sched_force;
            have = true;
        } else if (cfg.autotune && all_auto && cfg.schedule == DICOD_SCHED_EVENODD) {
            int64_t lmax = 0;
            for (int i = 0; i < n_sig; ++i)
                lmax = std::max(lmax, T[i] - W + 1);
            have = find_tuning(ctx, length_bucket(lmax), &e);
        }
        if (have) {
            cfg.colors = e.colors;
            cfg.update_cap = e.update_cap;
            m_tuned.resize(n_sig);
            for (int i = 0; i < n_sig; ++i)
                m_tuned[i] = T[i] >= W ? tuned_segments(T[i] - W + 1, W, e.colors, e.seg_len) : 0;
            n_seg = m_tuned.data();
            tuned = 1;
        }
    }

    Plan pl;
    int rc = make_plan(ctx, cfg.colors, n_sig, T, x_off, lam_in, n_seg, z_off, pl);
    if (rc != DICOD_OK)
        return rc;
    const int n_seg_tot = (int)pl.segs.size();
    const int64_t nL = pl.prefL[n_sig], nC = pl.prefC[n_sig], nA = pl.prefA[n_sig];
    const int64_t nN = pl.prefN[n_sig];
    const int n_kblk = check_kblocks(K, W);
    const int64_t max_ph = std::min<int64_t>(cfg.max_phases, (int64_t)1 << 22);

    // float rounds on the register-state kernel when the segments allow it
    const int cap_eff = effective_update_cap(cfg.update_cap, W);
    const bool reg_ok = !fp64 && cfg.reg_state != 0 && !pl.dicod &&
                        lgcd_wave_supported(K, pl.lm_max, cap_eff, false);
    const int box_cap = reg_ok ? std::max(cap_eff, 1) : 0;
    // free-running schedule: float rounds only, on the register-state kernel
    const bool async = cfg.schedule == DICOD_SCHED_ASYNC;
    if (async && (fp64 || !reg_ok))
        return fail(ctx, DICOD_ENOTSUP,
                    "the free-running schedule needs float rounds on the register-state kernel "
                    "(FP32 or MIXED, reg_state 1, segments of at most 256 positions, K <= 32, "
                    "update_cap in 1..64)");
    AsyncArgs ax;
    std::memset(&ax, 0, sizeof ax);
    if (async) {
        ax.sweeps = kAsyncSweeps;
        ax.ring_cap = lgcd_async_ring_cap(cap_eff, kAsyncSweeps);
        ax.n_teams = lgcd_async_teams(K, pl.lm_max, n_seg_tot, ctx->n_cu);
        if (ax.n_teams < 1)
            return fail(ctx, DICOD_ENOTSUP, "free-running schedule: no team fits the device");
        HIPCHECK(ctx, ensure(ws.ring, (size_t)2 * n_seg_tot * ax.ring_cap * sizeof(BoundaryRec)));
        HIPCHECK(ctx, ensure(ws.ring_wr, (size_t)4 * n_seg_tot * sizeof(uint32_t)));
    }
    HIPCHECK(ctx, ensure(ws.beta0, pl.zext * sizeof(double)));
    HIPCHECK(ctx, ensure(ws.g, pl.zext * (fp64 ? sizeof(double) : sizeof(float))));
    if (reg_ok) {
        HIPCHECK(ctx, ensure(ws.box, (size_t)2 * n_seg_tot * box_cap * sizeof(BoundaryRec)));
        HIPCHECK(ctx, ensure(ws.box_n, (size_t)2 * n_seg_tot * sizeof(uint32_t)));
        HIPCHECK(ctx, ensure(ws.z32, pl.zext * sizeof(float)));
    }
    HIPCHECK(ctx, ensure(ws.dirty, (pl.dicod ? 2 : 1) * n_seg_tot * sizeof(uint32_t)));
    HIPCHECK(ctx, ensure(ws.changed, (size_t)n_seg_tot * sizeof(uint32_t)));
    const int msg_cap = pl.dicod ? effective_update_cap(cfg.update_cap, W) : 0;
    if (pl.dicod) {
        HIPCHECK(ctx, ensure(ws.msg, (size_t)4 * n_seg_tot * msg_cap * sizeof(DicodMsg)));
        HIPCHECK(ctx, ensure(ws.msg_n, (size_t)4 * n_seg_tot * sizeof(uint32_t)));
    }
    HIPCHECK(ctx, ensure(ws.phase_upd, (size_t)(max_ph + 1) * sizeof(unsigned long long)));
    HIPCHECK(ctx, ensure(ws.sig_upd, n_sig * sizeof(unsigned long long)));
    HIPCHECK(ctx, ensure(ws.sig_last, n_sig * sizeof(int)));
    HIPCHECK(ctx, ensure(ws.counters, sizeof(Counters)));
    HIPCHECK(ctx, ensure(ws.nzmask, nN * sizeof(unsigned long long)));
    HIPCHECK(ctx, ensure(ws.part, (size_t)nC * n_kblk * kCheckParts * sizeof(double)));
    HIPCHECK(ctx, ensure(ws.results, n_sig * sizeof(CheckResult)));
    HIPCHECK(ctx, ensure(ws.lmax, n_sig * sizeof(unsigned long long)));
    HIPCHECK(ctx, ensure(ws.done, n_sig * sizeof(uint32_t)));
    if (cfg.trace_capacity > 0)
        HIPCHECK(ctx, ensure(ws.trace, cfg.trace_capacity * sizeof(dicod_trace_rec)));
    if (t_arena) {
        // everything a solve may need is carved before the first launch, so a
        // problem too large for the scratch fails before any work is queued
        if (!fp64 && cfg.fp64_polish_after > 0)
            HIPCHECK(ctx, ensure(ws.g64, pl.zext * sizeof(double)));
        if (ctx->cfg.precision == DICOD_PREC_MIXED) {
            HIPCHECK(ctx, ensure(ws.ebits, n_sig * sizeof(unsigned long long)));
            HIPCHECK(ctx, ensure(ws.thr, n_sig * sizeof(double)));
        }
        HIPCHECK(ctx, ensure(ws.sig, (size_t)n_sig * sizeof(SigDesc)));
        HIPCHECK(ctx, ensure(ws.segs, pl.segs.size() * sizeof(SegDesc)));
        for (int c = 0; c < pl.colors; ++c)
            HIPCHECK(ctx, ensure(ws.lists[c], pl.list[c].size() * sizeof(int32_t)));
        HIPCHECK(ctx, ensure(ws.tilesL, pl.prefL.size() * sizeof(int64_t)));
        HIPCHECK(ctx, ensure(ws.tilesC, pl.prefC.size() * sizeof(int64_t)));
        HIPCHECK(ctx, ensure(ws.tilesA, pl.prefA.size() * sizeof(int64_t)));
        HIPCHECK(ctx, ensure(ws.tilesN, pl.prefN.size() * sizeof(int64_t)));
        HIPCHECK(ctx, ensure(ws.slots, (size_t)n_sig * sizeof(int)));
        HIPCHECK(ctx, ensure(ws.lamin, (size_t)n_sig * sizeof(double)));
    }
    (void)box_cap;
    // pinned staging of the per-round uploads (descriptors, done flags): the
    // copies then leave the host at once; every use is separated from the next
    // by a synchronisation of the stream (the double check)
    const PinLayout pin = pin_layout(n_sig);
    const size_t pin_lam = pin.lam, pin_sig = pin.sig, pin_res = pin.res, pin_supd = pin.supd;
    const size_t pin_slast = pin.slast, pin_lbits = pin.lbits, pin_cnt = pin.cnt;
    const size_t pin_need = pin.need;
    const bool no_alloc = t_arena != nullptr;
    if (no_alloc && (pin_need > ctx->h_pin_cap || (size_t)(max_ph + 1) > ctx->h_upd_cap))
        return fail(ctx, DICOD_EINVAL, "pinned staging of the context is too small for this "
                                       "solve (one signal, max_phases of the configuration)");
    if (pin_need > ctx->h_pin_cap) {
        if (ctx->h_pin)
            (void)hipHostFree(ctx->h_pin);
        ctx->h_pin = nullptr;
        ctx->h_pin_cap = 0;
        HIPCHECK(ctx, hipHostMalloc((void**)&ctx->h_pin, pin_need, hipHostMallocDefault));
        ctx->h_pin_cap = pin_need;
    }
    auto upload_pinned = [&](DevBuf& b, const void* src, size_t bytes, size_t off) {
        hipError_t e = ensure(b, bytes);
        if (e != hipSuccess || bytes == 0)
            return e;
        std::memcpy(ctx->h_pin + off, src, bytes);
        return hipMemcpyAsync(b.p, ctx->h_pin + off, bytes, hipMemcpyHostToDevice, s);
    };
    if ((size_t)(max_ph + 1) > ctx->h_upd_cap) {
        if (ctx->h_upd)
            (void)hipHostFree(ctx->h_upd);
        ctx->h_upd = nullptr;
        ctx->h_upd_cap = 0;
        HIPCHECK(ctx, hipHostMalloc((void**)&ctx->h_upd,
                                    (size_t)(max_ph + 1) * sizeof(unsigned long long),
                                    hipHostMallocDefault));
        ctx->h_upd_cap = (size_t)(max_ph + 1);
    }
    HIPCHECK(ctx, upload_pinned(ws.sig, pl.sig.data(), (size_t)n_sig * sizeof(SigDesc), pin_sig));
    HIPCHECK(ctx, upload_cached(ws.segs, pl.segs, ws.sh_segs, s));
    for (int c = 0; c < pl.colors; ++c)
        HIPCHECK(ctx, upload_cached(ws.lists[c], pl.list[c], ws.sh_lists[c], s));
    HIPCHECK(ctx, upload_cached(ws.tilesL, pl.prefL, ws.sh_tL, s));
    HIPCHECK(ctx, upload_cached(ws.tilesC, pl.prefC, ws.sh_tC, s));
    HIPCHECK(ctx, upload_cached(ws.tilesA, pl.prefA, ws.sh_tA, s));
    HIPCHECK(ctx, upload_cached(ws.tilesN, pl.prefN, ws.sh_tN, s));

    hipEvent_t ev0 = pool_event(ctx, 0), ev1 = pool_event(ctx, 1);
    hipEvent_t ev2 = pool_event(ctx, 2), ev3 = pool_event(ctx, 3);
    if (!ev0 || !ev1 || !ev2 || !ev3)
        return fail(ctx, DICOD_EDEVICE, "hipEventCreate failed");
    HIPCHECK(ctx, hipEventRecord(ev0, s));

    // ---- 1. beta at Z = 0 ------------------------------------------------
    // FP64 and FP32 policies: double MFMA, and g starts equal to it (rounded
    // to float in FP32: the most accurate float start, which keeps the
    // double-precision finish short).  MIXED: the float state starts from a
    // cheaper float beta; the double beta0, needed only by the first
    // double-precision check, runs on a side stream meanwhile.
    const bool fast_init = ctx->cfg.precision == DICOD_PREC_MIXED;
    bool any_rel = false;
    for (int i = 0; i < n_sig; ++i)
        any_rel |= lam_in[i] < 0.0;
    if (!fast_init) {
        // the same pass zeroes Z (and its float copy) and takes lambda_max
        if (any_rel)
            HIPCHECK(ctx, launch_fill_u64(ws.lmax.as<unsigned long long>(), 0ull, n_sig, s));
        HIPCHECK(ctx, launch_corr_f64_x32(ctx->D64.as<double>(), K, P, W, dX,
                                          ws.sig.as<SigDesc>(), ws.tilesL.as<int64_t>(), n_sig,
                                          nL, ws.beta0.as<double>(),
                                          fp64 ? nullptr : ws.g.as<float>(),
                                          fp64 ? ws.g.as<double>() : nullptr, s, dZ,
                                          reg_ok ? ws.z32.as<float>() : nullptr,
                                          any_rel ? ws.lmax.as<unsigned long long>() : nullptr));
    } else {
        // the float start first; the double beta0 then runs beside the
        // descent (it is needed after the first float round only)
        HIPCHECK(ctx, launch_corr_bf16x3(ctx->Dsp.as<unsigned short>(), K, P, W, dX,
                                         ws.sig.as<SigDesc>(), ws.tilesL.as<int64_t>(), n_sig,
                                         nL, ws.g.as<float>(), s));
        HIPCHECK(ctx, hipEventRecord(ctx->ev_in, s));
        HIPCHECK(ctx, hipStreamWaitEvent(ctx->side, ctx->ev_in, 0));
        HIPCHECK(ctx, launch_corr_f64_x32(ctx->D64.as<double>(), K, P, W, dX,
                                          ws.sig.as<SigDesc>(), ws.tilesL.as<int64_t>(), n_sig,
                                          nL, ws.beta0.as<double>(), nullptr, nullptr,
                                          ctx->side));
        HIPCHECK(ctx, hipEventRecord(ctx->ev_beta, ctx->side));
    }
    bool beta_waited = !fast_init;
    // ---- descent state (queued behind the correlation, before the lambda
    // read-back, so that these small launches do not wait for the host) ----
    if (fast_init) {
        // Z = 0 over the union of the signals' [K][L] ranges (one launch per
        // contiguous run; the double correlation does it otherwise)
        std::vector<std::pair<int64_t, int64_t>> zr(n_sig);
        for (int i = 0; i < n_sig; ++i)
            zr[i] = {pl.sig[i].z_off, pl.sig[i].z_off + (int64_t)K * pl.sig[i].L};
        std::sort(zr.begin(), zr.end());
        int64_t lo = zr[0].first, hi = zr[0].second;
        for (int i = 1; i <= n_sig; ++i) {
            if (i < n_sig && zr[i].first <= hi) {
                hi = std::max(hi, zr[i].second);
                continue;
            }
            HIPCHECK(ctx, launch_fill_f64(dZ + lo, 0.0, (size_t)(hi - lo), s));
            if (reg_ok)  // float 0.0 is the all-zero word
                HIPCHECK(ctx, launch_fill_u32(ws.z32.as<uint32_t>() + lo, 0u,
                                              (size_t)(hi - lo), s));
            if (i < n_sig) {
                lo = zr[i].first;
                hi = zr[i].second;
            }
        }
    }
    HIPCHECK(ctx, launch_fill_u32(ws.dirty.as<uint32_t>(), 1u, n_seg_tot, s));
    HIPCHECK(ctx, launch_fill_u32(ws.changed.as<uint32_t>(), 1u, n_seg_tot, s));
    if (reg_ok)
        HIPCHECK(ctx, launch_fill_u32(ws.box_n.as<uint32_t>(), 0u, (size_t)2 * n_seg_tot, s));
    if (async)
        HIPCHECK(ctx, launch_fill_u32(ws.ring_wr.as<uint32_t>(), 0u, (size_t)4 * n_seg_tot, s));
    if (pl.dicod) {
        HIPCHECK(ctx, launch_fill_u32(ws.dirty.as<uint32_t>() + n_seg_tot, 0u, n_seg_tot, s));
        HIPCHECK(ctx, launch_fill_u32(ws.msg_n.as<uint32_t>(), 0u, (size_t)4 * n_seg_tot, s));
    }
    HIPCHECK(ctx, launch_fill_u64(ws.phase_upd.as<unsigned long long>(), 0ull, max_ph + 1, s));
    HIPCHECK(ctx, launch_fill_u64(ws.sig_upd.as<unsigned long long>(), 0ull, n_sig, s));
    HIPCHECK(ctx, launch_fill_u32(ws.done.as<uint32_t>(), 0u, n_sig, s));
    HIPCHECK(ctx, launch_fill_u32((uint32_t*)ws.sig_last.p, 0xffffffffu, n_sig, s));
    HIPCHECK(ctx, launch_fill_u64((unsigned long long*)ws.counters.p, 0ull,
                                  sizeof(Counters) / 8, s));
    // ---- 2. lambda --------------------------------------------------------
    std::vector<double> lmax(n_sig, 0.0);
    if (any_rel) {
        if (fast_init) {
            HIPCHECK(ctx, launch_fill_u64(ws.lmax.as<unsigned long long>(), 0ull, n_sig, s));
            // max of the split-bf16 beta, then the exact maximum over every
            // entry that the rounding error could make the maximum, recomputed
            // in double.  Per entry the error is at most
            // c sum |d| |x| <= c |D_k| |X[., t : t + W]| with
            // c = 3.1 2^-16 + (P W + 1) 2^-24 (bf16 unit roundoff 2^-8: the
            // dropped lo*lo product and the two representation remainders,
            // plus fp32 accumulation of P W terms and the final rounding), so
            // the maximiser's split value is at least v - 2 e, e = c max|D_k|
            // max_t |X[., t : t + W]| (5% margin on the bound).
            HIPCHECK(ctx, ensure(ws.ebits, n_sig * sizeof(unsigned long long)));
            HIPCHECK(ctx, ensure(ws.thr, n_sig * sizeof(double)));
            HIPCHECK(ctx, launch_fill_u64(ws.ebits.as<unsigned long long>(), 0ull, n_sig, s));
            HIPCHECK(ctx, launch_absmax_f32(ws.g.as<float>(), K, ws.sig.as<SigDesc>(),
                                            ws.tilesA.as<int64_t>(), n_sig, nA,
                                            ws.lmax.as<unsigned long long>(), s));
            HIPCHECK(ctx, launch_win_energy_max(dX, P, W, ws.sig.as<SigDesc>(),
                                                ws.tilesL.as<int64_t>(), n_sig, nL,
                                                ws.ebits.as<unsigned long long>(), s));
            HIPCHECK(ctx, launch_refine_threshold(ws.lmax.as<unsigned long long>(),
                                                  ws.ebits.as<unsigned long long>(), n_sig,
                                                  refine_coef(P, W, ctx->dnorm_max),
                                                  ws.thr.as<double>(), s));
            HIPCHECK(ctx, launch_fill_u64(ws.lmax.as<unsigned long long>(), 0ull, n_sig, s));
            HIPCHECK(ctx, launch_refine_absmax(ws.g.as<float>(), ctx->D64.as<double>(), dX, K, P,
                                               W, ws.sig.as<SigDesc>(), ws.tilesA.as<int64_t>(),
                                               n_sig, nA, ws.thr.as<double>(),
                                               ws.lmax.as<unsigned long long>(), s));
        }
        // lambda = |lambda_in| lambda_max, applied in the descriptors on the
        // device (no host round trip); the host forms the same values for the
        // statistics after the solve
        std::vector<int> ids(n_sig);
        for (int i = 0; i < n_sig; ++i)
            ids[i] = i;
        HIPCHECK(ctx, upload_cached(ws.slots, ids, ws.sh_slots, s));
        HIPCHECK(ctx, upload_pinned(ws.lamin, lam_in, (size_t)n_sig * sizeof(double), pin_lam));
        HIPCHECK(ctx, launch_apply_lambda(ws.sig.as<SigDesc>(), ws.slots.as<int>(),
                                          ws.lamin.as<double>(),
                                          ws.lmax.as<unsigned long long>(), n_sig, s));
    }
    HIPCHECK(ctx, hipEventRecord(ev1, s));

    // Precision of the descent state: float (FP32 policy) until the double
    // check has failed fp64_polish_after times, then double; always double in
    // the FP64 policy.
    bool cur64 = fp64;
    bool in_lds = false;
    if (!state_fits(pl, K, cur64, cfg.state_in_lds != 0, &in_lds))
        return fail(ctx, DICOD_ENOTSUP, "segments do not fit any phase kernel");
    if (pl.dicod && !in_lds)
        return fail(ctx, DICOD_ENOTSUP, "the DICOD schedule needs segments whose state fits LDS");
    bool polished = false, any_hbm = !in_lds && (cur64 || !reg_ok);

    PhaseArgs a;
    std::memset(&a, 0, sizeof a);
    a.segs = ws.segs.as<SegDesc>();
    a.Z = dZ;
    a.sigs = ws.sig.as<SigDesc>();
    a.K = K;
    a.W = W;
    // update_cap 0 means "run each segment to local convergence"; a finite
    // bound still guarantees that every workgroup exits.
    a.cap = effective_update_cap(cfg.update_cap, W);
    a.dirty = ws.dirty.as<uint32_t>();
    a.phase_upd = ws.phase_upd.as<unsigned long long>();
    a.sig_upd = ws.sig_upd.as<unsigned long long>();
    a.sig_last_upd = ws.sig_last.as<int>();
    a.counters = ws.counters.as<Counters>();
    a.trace = cfg.trace_capacity > 0 ? ws.trace.as<dicod_trace_rec>() : nullptr;
    a.trace_cap = cfg.trace_capacity;
    a.lm_max = pl.lm_max;
    a.lext_max = pl.lext_max;
    a.dicod = pl.dicod ? 1 : 0;
    a.n_seg = n_seg_tot;
    a.msg_cap = msg_cap;
    a.msg = pl.dicod ? ws.msg.as<DicodMsg>() : nullptr;
    a.msg_n = pl.dicod ? ws.msg_n.as<uint32_t>() : nullptr;
    a.box = reg_ok ? ws.box.as<BoundaryRec>() : nullptr;
    a.box_n = reg_ok ? ws.box_n.as<uint32_t>() : nullptr;
    a.box_cap = box_cap;
    a.z32 = reg_ok ? ws.z32.as<float>() : nullptr;
    a.changed = ws.changed.as<uint32_t>();
    a.phase_stride = 0;
    if (async) {
        ax.ring = ws.ring.as<BoundaryRec>();
        ax.ring_w = ws.ring_wr.as<uint32_t>();
        ax.ring_r = ws.ring_wr.as<uint32_t>() + (size_t)2 * n_seg_tot;
    }
    auto set_state = [&](bool use64, bool lds) {
        a.g = use64 && !fp64 ? ws.g64.p : ws.g.p;
        a.S = use64 ? (lds ? ctx->St64.p : ctx->S64.p) : (lds ? ctx->St32.p : ctx->S32.p);
        a.n2 = use64 ? ctx->n2_64.p : ctx->n2_32.p;
        a.inv_n2 = use64 ? ctx->inv64.p : ctx->inv32.p;
        for (int i = 0; i < n_sig; ++i)
            pl.sig[i].eps_stop = use64 ? eps : eps * cfg.inner_eps_factor;
        return launch_set_eps_stop(ws.sig.as<SigDesc>(), n_sig,
                                   use64 ? eps : eps * cfg.inner_eps_factor, s);
    };
    HIPCHECK(ctx, set_state(cur64, in_lds));

    int64_t phase = 0, n_launch = 0, conv_phase = -1;
    int n_refresh = 0, round = 0;
    int n_checks = 0, last_out = 0;  // checks run; state buffer the last refresh wrote
    bool accepted = false, out_of_phases = false;
    double t_cd = 0.0, t_verify = 0.0, t_kernel = 0.0;
    int64_t round_upd[4] = {0, 0, 0, 0}, round_ph[4] = {0, 0, 0, 0};
    int64_t round_launch[4] = {0, 0, 0, 0};
    double round_ms[4] = {0.0, 0.0, 0.0, 0.0}, round_kms[4] = {0.0, 0.0, 0.0, 0.0};
    int round_state[4] = {0, 0, 0, 0};
    std::vector<CheckResult> res(n_sig);
    std::vector<uint32_t> done(n_sig, 0u);
    std::vector<double> round_mdz((size_t)n_sig * 4, 0.0);
    // phases queued past a round's convergence apply nothing: they are not
    // counted in n_phases (round r starts at phase r_start[r]; r_over[r]
    // overshoot phases ran before it)
    std::vector<int64_t> r_start, r_over;
    int64_t overshoot = 0;

    for (;;) {
        // ---- 3. coloured phases until C consecutive phases apply nothing
        HIPCHECK(ctx, hipEventRecord(ev2, s));
        const int64_t start = phase;
        r_start.push_back(start);
        r_over.push_back(overshoot);
        const int64_t launch0 = n_launch;
        const double kern0 = t_kernel;
        conv_phase = -1;
        // Chunks of phases_per_poll phases; each chunk's update counts are
        // copied to the host behind it.  Without per-launch timing the next
        // chunk is queued before the host waits for the previous chunk's
        // counts, so the device does not idle on the poll; phases queued after
        // convergence find no dirty segment and apply nothing.
        const bool overlap = !cfg.timing;
        // a free-running float round: every launch runs all segments, and one
        // launch that applies nothing ends the round (no record is left: a
        // segment with records waiting runs and applies them)
        const bool async_round = async && !cur64;
        const int quiet_n = async_round ? 1 : pl.colors;
        int64_t checked = start + quiet_n - 1;    // next phase whose quiet window is tested
        int64_t copied = start;                   // counts copied (or queued) below this
        int64_t known = start;                    // counts on the host below this
        int64_t q_end[2] = {0, 0};                // queued chunks (FIFO of at most 2)
        int q_head = 0, nq = 0;
        size_t evi = 4;
        bool limit = false;
        for (;;) {
            bool launched = false;
            if (phase >= max_ph || (!cur64 && phase - start >= kRoundPhaseLimit)) {
                // In float, rounding noise near the stop threshold can keep a
                // few coordinates changing for ever; after a bounded number of
                // phases the double-precision test decides instead.
                limit = true;
            } else {
                const int64_t chunk = std::min<int64_t>(
                    async_round ? std::min(cfg.phases_per_poll, 2) : cfg.phases_per_poll,
                    max_ph - phase);
                evi = 4;
                for (int64_t c = 0; c < chunk; ++c, ++phase) {
                    const int par = (int)(phase % pl.colors);
                    a.list = ws.lists[par].as<int32_t>();
                    a.n_list = (int)pl.list[par].size();
                    a.phase = (int)phase;
                    if (a.n_list == 0 && !async_round)
                        continue;
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    if (cfg.timing) {
                        e0 = pool_event(ctx, evi++);
                        e1 = pool_event(ctx, evi++);
                        if (!e0 || !e1)
                            return fail(ctx, DICOD_EDEVICE, "hipEventCreate failed");
                        HIPCHECK(ctx, hipEventRecord(e0, s));
                    }
                    size_t lds = 0;
                    const bool use_reg = !cur64 && reg_ok;
                    hipError_t e = async_round ? launch_lgcd_async(a, ax, s)
                                   : use_reg   ? launch_lgcd_wave(a, s)
                                   : in_lds    ? launch_lgcd_phase(a, cur64, &lds, s)
                                               : launch_lgcd_phase_gm(a, cur64, &lds, s);
                    if (e != hipSuccess)
                        return fail(ctx, DICOD_EDEVICE,
                                    "LGCD phase launch (%s state, %zu bytes LDS): %s",
                                    use_reg ? "register" : in_lds ? "LDS" : "HBM", lds,
                                    hipGetErrorString(e));
                    ++n_launch;
                    if (cfg.timing)
                        HIPCHECK(ctx, hipEventRecord(e1, s));
                }
                HIPCHECK(ctx, hipMemcpyAsync(ctx->h_upd + copied,
                                             ws.phase_upd.as<unsigned long long>() + copied,
                                             (size_t)(phase - copied) * sizeof(unsigned long long),
                                             hipMemcpyDeviceToHost, s));
                copied = phase;
                const int tail = (q_head + nq) & 1;
                q_end[tail] = copied;
                HIPCHECK(ctx, hipEventRecord(ctx->ev_poll[tail], s));
                ++nq;
                launched = true;
            }
            // wait for the oldest chunks, keeping one in flight while phases
            // are still being queued
            while (nq > (launched && overlap ? 1 : 0)) {
                HIPCHECK(ctx, hipEventSynchronize(ctx->ev_poll[q_head]));
                known = q_end[q_head];
                q_head ^= 1;
                --nq;
                if (cfg.timing)
                    for (size_t i = 4; i < evi; i += 2)
                        t_kernel += elapsed_ms(ctx->ev_pool[i], ctx->ev_pool[i + 1]);
            }
            // converged once `colors` consecutive phases applied nothing
            for (int64_t p = checked; p < known; ++p) {
                bool quiet = true;
                for (int c = 0; c < quiet_n; ++c)
                    quiet &= ctx->h_upd[p - c] == 0;
                if (quiet) {
                    conv_phase = p;
                    break;
                }
            }
            checked = std::max(checked, known);
            if (conv_phase >= 0 || (limit && nq == 0))
                break;
        }
        if (conv_phase < 0 && phase >= max_ph)
            out_of_phases = true;
        HIPCHECK(ctx, hipEventRecord(ev3, s));
        HIPCHECK(ctx, hipEventSynchronize(ev3));
        const double t_round = elapsed_ms(ev2, ev3);
        t_cd += t_round;
        if (conv_phase >= 0)
            overshoot += phase - (conv_phase + 1);
        if (round < 4) {
            round_ms[round] = t_round;
            const int64_t last = conv_phase >= 0 ? conv_phase + 1 : phase;
            round_ph[round] = last - start;
            round_launch[round] = n_launch - launch0;
            round_kms[round] = t_kernel - kern0;
            round_state[round] = (cur64 ? 1 : 0) | (in_lds ? 0 : 2) |
                                 (!cur64 && reg_ok ? 4 : 0) | (async_round ? 8 : 0);
            for (int64_t p = start; p < last; ++p)
                round_upd[round] += (int64_t)ctx->h_upd[p];
        }
        ++round;

        // ---- 4. double-precision stop test; refresh of the next round's g
        const bool next64 = cur64 || (cfg.fp64_polish_after > 0 &&
                                      n_refresh + 1 >= cfg.fp64_polish_after);
        bool next_lds = in_lds;
        if (next64 != cur64 && (!state_fits(pl, K, true, cfg.state_in_lds != 0, &next_lds) ||
                                (pl.dicod && !next_lds)))
            return fail(ctx, DICOD_ENOTSUP, "segments do not fit the double-state kernel");
        if (next64 && !fp64)
            HIPCHECK(ctx, ensure(ws.g64, pl.zext * sizeof(double)));
        void* g_next = next64 && !fp64 ? ws.g64.p : ws.g.p;
        const double flag_eps = next64 ? eps : eps * cfg.inner_eps_factor;
        HIPCHECK(ctx, hipEventRecord(ev2, s));
        if (!beta_waited) {
            HIPCHECK(ctx, hipStreamWaitEvent(s, ctx->ev_beta, 0));
            beta_waited = true;
        }
        // After a double round the maintained state is exact to rounding, and
        // the stop test reads it directly; otherwise g is recomputed from Z.
        const double* g_in = (cur64 && !cfg.verify_from_scratch)
                                 ? (fp64 ? ws.g.as<double>() : ws.g64.as<double>())
                                 : nullptr;
        // Only the tiles within reach of a segment whose Z changed since the
        // last check are recomputed when that check wrote the same state
        // buffer, or this one writes none (the check of a maintained double
        // state after a double round, which changed few segments).
        const int out_kind = g_in ? 0 : next64 ? 2 : 1;
        const bool skip_tiles = n_checks > 0 && (out_kind == 0 || out_kind == last_out);
        if (!g_in)
            HIPCHECK(ctx, launch_nz_mask(dZ, ws.sig.as<SigDesc>(), ws.tilesN.as<int64_t>(), n_sig,
                                         K, nN, ws.nzmask.as<unsigned long long>(), s));
        HIPCHECK(ctx, launch_grad_check(dX, ws.beta0.as<double>(), dZ,
                                        ws.nzmask.as<unsigned long long>(),
                                        ctx->Sc64.as<double>(), ctx->n2_64.as<double>(), K, P, W,
                                        ws.sig.as<SigDesc>(), ws.tilesC.as<int64_t>(), n_sig, nC,
                                        flag_eps, ws.done.as<uint32_t>(),
                                        ws.dirty.as<uint32_t>(), g_in ? nullptr : g_next, next64,
                                        g_in, ws.part.as<double>(),
                                        reg_ok && !next64 && !g_in ? ws.z32.as<float>() : nullptr,
                                        skip_tiles ? ws.changed.as<uint32_t>() : nullptr, s));
        HIPCHECK(ctx, launch_fill_u32(ws.changed.as<uint32_t>(), 0u, n_seg_tot, s));
        ++n_checks;
        if (out_kind != 0)
            last_out = out_kind;
        HIPCHECK(ctx, launch_check_reduce(ws.part.as<double>(), ws.tilesC.as<int64_t>(), nC,
                                          n_kblk, n_sig, ws.results.as<CheckResult>(), s));
        HIPCHECK(ctx, hipMemcpyAsync(ctx->h_pin + pin_res, ws.results.p,
                                     n_sig * sizeof(CheckResult), hipMemcpyDeviceToHost, s));
        HIPCHECK(ctx, hipEventRecord(ev3, s));
        HIPCHECK(ctx, hipEventSynchronize(ev3));
        std::memcpy(res.data(), ctx->h_pin + pin_res, n_sig * sizeof(CheckResult));
        t_verify += elapsed_ms(ev2, ev3);
        if (round <= 4)
            for (int i = 0; i < n_sig; ++i)
                if (!done[i])
                    round_mdz[(size_t)i * 4 + (round - 1)] = res[i].max_dz;
        accepted = true;
        for (int i = 0; i < n_sig; ++i) {
            done[i] = res[i].max_dz < eps ? 1u : 0u;
            accepted &= done[i] != 0u;
        }
        if (accepted || out_of_phases || n_refresh >= cfg.max_refresh)
            break;
        // Signals that passed are frozen; the others had g refreshed and their
        // offending segments marked dirty.  Resuming on colour 0 keeps a
        // signal's sequence of segment runs independent of its co-runners.
        ++n_refresh;
        if (next64 != cur64) {
            cur64 = true;
            in_lds = next_lds;
            polished = true;
            any_hbm |= !in_lds;
        }
        HIPCHECK(ctx, set_state(cur64, in_lds));
        HIPCHECK(ctx, upload_pinned(ws.done, done.data(), (size_t)n_sig * sizeof(uint32_t), 0));
        // a signal that passed is frozen: the check may have flagged its
        // segments against the next round's tighter threshold
        HIPCHECK(ctx, launch_clear_done_dirty(ws.segs.as<SegDesc>(), n_seg_tot,
                                              ws.done.as<uint32_t>(), ws.dirty.as<uint32_t>(),
                                              s));
        if (reg_ok)  // records of the last round are stale: g was refreshed
            HIPCHECK(ctx, launch_fill_u32(ws.box_n.as<uint32_t>(), 0u, (size_t)2 * n_seg_tot, s));
        if (async)
            HIPCHECK(ctx, launch_fill_u32(ws.ring_wr.as<uint32_t>(), 0u, (size_t)4 * n_seg_tot,
                                          s));
        while (phase % pl.colors)
            ++phase;
        if (pl.dicod) {
            // the next round reads the flags of parity 0 (set by the check) and
            // no message of the previous round
            phase += phase & 1;
            HIPCHECK(ctx, launch_fill_u32(ws.dirty.as<uint32_t>() + n_seg_tot, 0u, n_seg_tot, s));
            HIPCHECK(ctx, launch_fill_u32(ws.msg_n.as<uint32_t>(), 0u, (size_t)4 * n_seg_tot, s));
        }
    }

    std::vector<unsigned long long> supd(n_sig);
    std::vector<int> slast(n_sig);
    Counters cnt;
    HIPCHECK(ctx, hipMemcpyAsync(ctx->h_pin + pin_supd, ws.sig_upd.p,
                                 n_sig * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->h_pin + pin_slast, ws.sig_last.p, n_sig * sizeof(int),
                                 hipMemcpyDeviceToHost, s));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->h_pin + pin_cnt, ws.counters.p, sizeof cnt,
                                 hipMemcpyDeviceToHost, s));
    std::vector<unsigned long long> lbits(n_sig, 0ull);
    if (any_rel)
        HIPCHECK(ctx, hipMemcpyAsync(ctx->h_pin + pin_lbits, ws.lmax.p,
                                     n_sig * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHECK(ctx, hipStreamSynchronize(s));
    std::memcpy(supd.data(), ctx->h_pin + pin_supd, n_sig * sizeof(unsigned long long));
    std::memcpy(slast.data(), ctx->h_pin + pin_slast, n_sig * sizeof(int));
    std::memcpy(&cnt, ctx->h_pin + pin_cnt, sizeof cnt);
    if (any_rel)
        std::memcpy(lbits.data(), ctx->h_pin + pin_lbits, n_sig * sizeof(unsigned long long));
    ctx->last_trace_n = (int64_t)cnt.trace_n;
    if (cnt.box_overflow)
        return fail(ctx, DICOD_EDEVICE,
                    "internal: %llu boundary records found a full mailbox or ring",
                    (unsigned long long)cnt.box_overflow);
    for (int i = 0; any_rel && i < n_sig; ++i) {
        // the arithmetic of k_apply_lambda
        double v;
        std::memcpy(&v, &lbits[i], sizeof v);
        lmax[i] = v;
        if (lam_in[i] < 0.0) {
            pl.sig[i].lam = -lam_in[i] * v;
            if (!(pl.sig[i].lam > 0.0))
                pl.sig[i].lam = 1e-300;  // X orthogonal to every atom: Z = 0
        }
    }
    // Duality gap of the returned Z (Gap Safe rule): theta = R / max(lambda,
    // max |D^T R|) is dual feasible, gap = E(Z) - Dual(theta) with
    // Dual(theta) = -lambda^2 |R|^2 / (2 s^2) + lambda <R, X> / s and
    // <R, X> = |X|^2 - <beta0, Z>.  With screen = 1 the coordinates the
    // sphere rule proves zero are counted from g recomputed in double.
    std::vector<double> gap(n_sig, 0.0), rule(2 * (size_t)n_sig, 0.0);
    std::vector<unsigned long long> n_scr(n_sig, 0ull);
    for (int i = 0; i < n_sig; ++i) {
        const double lam = pl.sig[i].lam;
        const double sc = std::max(lam, res[i].gmax);
        const double primal = 0.5 * res[i].sum_r2 + lam * res[i].l1;
        const double dual =
            -lam * lam * res[i].sum_r2 / (2.0 * sc * sc) + lam * (res[i].x2 - res[i].bx) / sc;
        gap[i] = std::max(primal - dual, 0.0);
        rule[2 * i] = 1.0 / sc;
        rule[2 * i + 1] = std::sqrt(2.0 * gap[i]) / lam;
    }
    if (cfg.screen) {
        if (!fp64)
            HIPCHECK(ctx, ensure(ws.g64, pl.zext * sizeof(double)));
        void* gs = fp64 ? ws.g.p : ws.g64.p;
        HIPCHECK(ctx, launch_nz_mask(dZ, ws.sig.as<SigDesc>(), ws.tilesN.as<int64_t>(), n_sig, K,
                                     nN, ws.nzmask.as<unsigned long long>(), s));
        HIPCHECK(ctx, launch_grad_check(dX, ws.beta0.as<double>(), dZ,
                                        ws.nzmask.as<unsigned long long>(),
                                        ctx->Sc64.as<double>(), ctx->n2_64.as<double>(), K, P, W,
                                        ws.sig.as<SigDesc>(), ws.tilesC.as<int64_t>(), n_sig, nC,
                                        eps, nullptr, nullptr, gs, true, nullptr,
                                        ws.part.as<double>(), nullptr, nullptr, s));
        HIPCHECK(ctx, upload(ws.thr, rule, s));
        HIPCHECK(ctx, ensure(ws.ebits, n_sig * sizeof(unsigned long long)));
        HIPCHECK(ctx, launch_fill_u64(ws.ebits.as<unsigned long long>(), 0ull, n_sig, s));
        HIPCHECK(ctx, launch_screen_count(gs, true, ctx->n2_64.as<double>(), K,
                                          ws.sig.as<SigDesc>(), ws.tilesA.as<int64_t>(), n_sig,
                                          nA, ws.thr.as<double>(),
                                          ws.ebits.as<unsigned long long>(), s));
        HIPCHECK(ctx, hipMemcpyAsync(n_scr.data(), ws.ebits.p, n_sig * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost, s));
        HIPCHECK(ctx, hipStreamSynchronize(s));
    }
    const double t_init = elapsed_ms(ev0, ev1);
    const double t_total = now_ms() - t_call0;
    if (st) {
        for (int i = 0; i < n_sig; ++i) {
            dicod_stats& o = st[i];
            std::memset(&o, 0, sizeof o);
            o.n_updates = (int64_t)supd[i];
            {
                // phase index without the overshoot of earlier rounds
                auto strip = [&](int64_t ph) {
                    size_t r = 0;
                    while (r + 1 < r_start.size() && r_start[r + 1] <= ph)
                        ++r;
                    return r < r_over.size() ? ph - r_over[r] : ph;
                };
                const int64_t last_ph = conv_phase >= 0 ? conv_phase + 1 : phase;
                o.n_phases = n_sig == 1 ? strip(last_ph)
                                        : std::min<int64_t>(strip(last_ph),
                                                            strip((int64_t)slast[i]) + 3);
            }
            o.n_phase_launches = n_launch;
            o.n_segment_runs = (int64_t)cnt.seg_runs;
            o.nnz = (int64_t)res[i].nnz;
            o.n_seg = pl.sig[i].M;
            o.seg_len = (int)(pl.sig[i].L / pl.sig[i].M);
            o.converged = res[i].max_dz < eps ? 1 : 0;
            o.n_refresh = n_refresh;
            o.lambda = pl.sig[i].lam;
            o.lambda_max = lmax[i];
            o.eps = eps;
            o.objective = 0.5 * res[i].sum_r2 + pl.sig[i].lam * res[i].l1;
            o.max_dz = res[i].max_dz;
            o.kkt_on = res[i].kkt_on;
            o.kkt_off = res[i].kkt_off;
            o.max_abs_z = res[i].max_abs_z;
            o.t_init_ms = t_init;
            o.t_cd_ms = t_cd;
            o.t_verify_ms = t_verify;
            o.t_total_ms = t_total;
            o.t_lgcd_kernel_ms = t_kernel;
            for (int r = 0; r < 4; ++r) {
                o.round_max_dz[r] = round_mdz[(size_t)i * 4 + r];
                o.round_updates[r] = round_upd[r];
                o.round_phases[r] = round_ph[r];
                o.round_ms[r] = round_ms[r];
                o.round_kernel_ms[r] = round_kms[r];
                o.round_launches[r] = round_launch[r];
                o.round_state[r] = round_state[r];
            }
            o.state_in_hbm = any_hbm ? 1 : 0;
            o.polished_fp64 = polished ? 1 : 0;
            o.duality_gap = gap[i];
            o.n_screened = cfg.screen ? (int64_t)n_scr[i] : -1;
            o.colors = pl.colors;
            o.update_cap = cfg.update_cap == 0 ? 0 : effective_update_cap(cfg.update_cap, W);
            o.tuned = tuned;
        }
    }
    if (!accepted)
        return fail(ctx, DICOD_ENOTCONV,
                    out_of_phases ? "max_phases reached before the stop test held"
                                  : "double-precision stop test failed after max_refresh "
                                    "refreshes");
    return DICOD_OK;
}

}  // namespace dicod

// ---------------------------------------------------------------------------
// public solve entry points
// ---------------------------------------------------------------------------
extern "C" int dicod_solve_device(dicod_ctx* ctx, const float* X_dev, int64_t T,
                                  double lambda, double eps, int n_seg, double* Z_dev,
                                  dicod_stats* st, void* stream)
{
    if (!ctx)
        return DICOD_EINVAL;
    ctx->err.clear();
    HIPCHECK(ctx, hipSetDevice(ctx->cfg.device));
    const int64_t zero = 0;
    return solve_device_batch(ctx, 1, X_dev, &T, &zero, &lambda, eps, &n_seg, Z_dev, &zero,
                              st, stream ? (hipStream_t)stream : ctx->stream);
}

extern "C" int dicod_solve_device_noalloc(dicod_ctx* ctx, const float* X_dev, int64_t T,
                                          double lambda, double eps, int n_seg, double* Z_dev,
                                          dicod_stats* st, void* stream)
{
    if (!ctx)
        return DICOD_EINVAL;
    ctx->err.clear();
    if (!ctx->scratch)
        return fail(ctx, DICOD_EDEVICE, "dicod_solve_device_noalloc: no static scratch");
    if (ctx->cfg.timing)
        return fail(ctx, DICOD_EINVAL, "dicod_solve_device_noalloc: timing = 1 needs events "
                                       "per launch; not available without allocation");
    HIPCHECK(ctx, hipSetDevice(ctx->cfg.device));
    // the views of the previous call are stale: this call lays the scratch out
    // for its own problem, and uploads nothing from the plan cache
    ctx->ws_scratch = Workspace();
    Arena ar;
    ar.base = static_cast<unsigned char*>(ctx->scratch);
    ar.cap = dicod::scratch_bytes();
    t_arena = &ar;
    const int64_t zero = 0;
    int rc = solve_device_batch(ctx, 1, X_dev, &T, &zero, &lambda, eps, &n_seg, Z_dev, &zero,
                                st, stream ? (hipStream_t)stream : ctx->stream);
    t_arena = nullptr;
    if (ar.overflow)
        rc = fail(ctx, DICOD_EINVAL,
                  "dicod_solve_device_noalloc: this problem needs %zu bytes of scratch; the "
                  "static scratch holds %zu bytes (use dicod_solve_device)", ar.need, ar.cap);
    return rc;
}

extern "C" int dicod_solve_batch_device(dicod_ctx* ctx, int n_sig, const float* X_dev,
                                        const int64_t* T, const int64_t* x_off,
                                        const double* lambda, double eps, const int* n_seg,
                                        double* Z_dev, const int64_t* z_off,
                                        dicod_stats* st, void* stream)
{
    if (!ctx)
        return DICOD_EINVAL;
    ctx->err.clear();
    HIPCHECK(ctx, hipSetDevice(ctx->cfg.device));
    return solve_device_batch(ctx, n_sig, X_dev, T, x_off, lambda, eps, n_seg, Z_dev, z_off,
                              st, stream ? (hipStream_t)stream : ctx->stream);
}

extern "C" int dicod_solve(dicod_ctx* ctx, const float* X, int P, int64_t T, const float* D,
                           int K, int W, double lambda, double eps, int n_seg, double* Z_out,
                           dicod_stats* st)
{
    if (!ctx)
        return DICOD_EINVAL;
    ctx->err.clear();
    if (!X || !Z_out)
        return fail(ctx, DICOD_EINVAL, "dicod_solve: X or Z_out is NULL");
    if (P <= 0 || K <= 0 || W <= 0)
        return fail(ctx, DICOD_EINVAL, "dicod_solve: K=%d P=%d W=%d must be > 0", K, P, W);
    if (T < W)
        return fail(ctx, DICOD_EINVAL, "dicod_solve: T=%lld < W=%d", (long long)T, W);
    if (D) {
        int rc = dicod_set_dictionary(ctx, D, K, P, W);
        if (rc != DICOD_OK)
            return rc;
    } else if (!ctx->has_dict || ctx->K != K || ctx->P != P || ctx->W != W) {
        return fail(ctx, DICOD_EINVAL,
                    "dicod_solve: D is NULL and the resident dictionary does not match");
    }
    const size_t nx = (size_t)P * T;
    for (size_t i = 0; i < nx; ++i)
        if (!std::isfinite(X[i]))
            return fail(ctx, DICOD_EINVAL, "dicod_solve: X[%zu] is not finite", i);
    HIPCHECK(ctx, hipSetDevice(ctx->cfg.device));
    const int64_t L = T - W + 1;
    const size_t nz = (size_t)K * L;
    HIPCHECK(ctx, ensure(ctx->ws.X, nx * sizeof(float)));
    HIPCHECK(ctx, ensure(ctx->ws.Zout, nz * sizeof(double)));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->ws.X.p, X, nx * sizeof(float), hipMemcpyHostToDevice,
                                 ctx->stream));
    const int64_t zero = 0;
    int rc = solve_device_batch(ctx, 1, ctx->ws.X.as<float>(), &T, &zero, &lambda, eps, &n_seg,
                                ctx->ws.Zout.as<double>(), &zero, st, ctx->stream);
    if (rc == DICOD_OK || rc == DICOD_ENOTCONV) {
        hipError_t e = hipMemcpy(Z_out, ctx->ws.Zout.p, nz * sizeof(double),
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return fail(ctx, DICOD_EDEVICE, "copy of Z: %s", hipGetErrorString(e));
    }
    return rc;
}

extern "C" int dicod_correlate(dicod_ctx* ctx, const float* X, int64_t T, int precision,
                               double* out)
{
    if (!ctx)
        return DICOD_EINVAL;
    ctx->err.clear();
    if (!X || !out)
        return fail(ctx, DICOD_EINVAL, "dicod_correlate: NULL argument");
    if (!ctx->has_dict)
        return fail(ctx, DICOD_EINVAL, "dicod_correlate: no resident dictionary");
    const int K = ctx->K, P = ctx->P, W = ctx->W;
    if (T < W)
        return fail(ctx, DICOD_EINVAL, "dicod_correlate: T < W");
    if (precision != DICOD_PREC_FP64 && precision != DICOD_PREC_MIXED)
        return fail(ctx, DICOD_EINVAL, "dicod_correlate: precision %d is not FP64 or MIXED",
                    precision);
    HIPCHECK(ctx, hipSetDevice(ctx->cfg.device));
    hipStream_t s = ctx->stream;
    const int64_t L = T - W + 1;
    std::vector<SigDesc> sd(1);
    sd[0].x_off = 0;
    sd[0].z_off = 0;
    sd[0].T = T;
    sd[0].L = L;
    sd[0].seg_base = 0;
    sd[0].M = 1;
    sd[0].lam = 0.0;
    std::vector<int64_t> pref = {0, ceil_div(L, kTile)};
    DevBuf dx, dout, dsig, dpref;
    HIPCHECK(ctx, ensure(dx, (size_t)P * T * sizeof(float)));
    HIPCHECK(ctx, ensure(dout, (size_t)K * L * sizeof(double)));
    HIPCHECK(ctx, upload(dsig, sd, s));
    HIPCHECK(ctx, upload(dpref, pref, s));
    HIPCHECK(ctx, hipMemcpyAsync(dx.p, X, (size_t)P * T * sizeof(float), hipMemcpyHostToDevice, s));
    if (precision == DICOD_PREC_MIXED) {
        HIPCHECK(ctx, launch_corr_bf16x3(ctx->Dsp.as<unsigned short>(), K, P, W, dx.as<float>(),
                                         dsig.as<SigDesc>(), dpref.as<int64_t>(), 1, pref[1],
                                         dout.as<float>(), s));
        std::vector<float> o32((size_t)K * L);
        HIPCHECK(ctx, hipMemcpyAsync(o32.data(), dout.p, o32.size() * sizeof(float),
                                     hipMemcpyDeviceToHost, s));
        HIPCHECK(ctx, hipStreamSynchronize(s));
        for (size_t i = 0; i < o32.size(); ++i)
            out[i] = (double)o32[i];
        return DICOD_OK;
    }
    HIPCHECK(ctx, launch_corr_f64_x32(ctx->D64.as<double>(), K, P, W, dx.as<float>(),
                                      dsig.as<SigDesc>(), dpref.as<int64_t>(), 1, pref[1],
                                      dout.as<double>(), nullptr, nullptr, s));
    HIPCHECK(ctx, hipMemcpyAsync(out, dout.p, (size_t)K * L * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    HIPCHECK(ctx, hipStreamSynchronize(s));
    return DICOD_OK;
}

extern "C" int dicod_get_trace(dicod_ctx* ctx, dicod_trace_rec* out, int64_t cap, int64_t* n)
{
    if (!ctx)
        return DICOD_EINVAL;
    if (!n || (cap > 0 && !out))
        return fail(ctx, DICOD_EINVAL, "dicod_get_trace: NULL argument");
    if (ctx->cfg.trace_capacity <= 0)
        return fail(ctx, DICOD_EINVAL, "dicod_get_trace: trace_capacity is 0");
    int64_t avail = std::min<int64_t>(ctx->last_trace_n, ctx->cfg.trace_capacity);
    *n = avail;
    int64_t cnt = std::min<int64_t>(avail, cap);
    if (cnt > 0) {
        HIPCHECK(ctx, hipSetDevice(ctx->cfg.device));
        HIPCHECK(ctx, hipMemcpy(out, ctx->ws.trace.p, (size_t)cnt * sizeof(dicod_trace_rec),
                                hipMemcpyDeviceToHost));
    }
    return DICOD_OK;
}

// ---------------------------------------------------------------------------
// serving (dicod_serve.cpp)
// ---------------------------------------------------------------------------
extern "C" int dicod_submit(dicod_ctx* ctx, const float* X, int64_t T, double lambda,
                            double eps, int n_seg, uint64_t* req_id)
{
    if (!ctx)
        return DICOD_EINVAL;
    return dicod::server_submit(ctx, X, T, lambda, eps, n_seg, req_id);
}

extern "C" int dicod_poll(dicod_ctx* ctx, uint64_t req_id, double* Z_out, dicod_stats* st)
{
    if (!ctx)
        return DICOD_EINVAL;
    return dicod::server_poll(ctx, req_id, Z_out, st);
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
namespace {

bool find_tuning(const dicod_ctx* ctx, int bucket, dicod_tune_entry* e)
{
    auto it = ctx->tuning.find(bucket);
    if (it == ctx->tuning.end() || it->second.K != ctx->K || it->second.P != ctx->P ||
        it->second.W != ctx->W)
        return false;
    *e = it->second;
    return true;
}

int team_threads_for(int K, int seg_len, int cap)
{
    if (!lgcd_wave_supported(K, seg_len, cap, false))
        return 0;
    return seg_len <= 64 ? 64 : seg_len <= 128 ? 128 : 256;
}

// Candidate longest-segment lengths for C colours: the shortest legal one,
// the register kernel's team boundaries, and multiples of W.
std::vector<int> seg_ladder(int W, int C, int64_t lmax)
{
    const int lo = (int)min_segment(W, C);
    std::vector<int> v = {lo, 64, 96, 128, 192, 256, 2 * W, 3 * W, 4 * W, 8 * W};
    std::vector<int> out;
    for (int x : v)
        if (x >= lo && x <= lmax)
            out.push_back(x);
    if (out.empty())
        out.push_back((int)std::min<int64_t>(lmax, INT32_MAX));
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    return out;
}

}  // namespace

extern "C" int dicod_autotune_device(dicod_ctx* ctx, int n_sig, const float* X_dev,
                                     const int64_t* T, const int64_t* x_off,
                                     const double* lambda, double eps, double* Z_dev,
                                     const int64_t* z_off, int max_trials,
                                     dicod_tune_entry* out)
{
    if (!ctx)
        return DICOD_EINVAL;
    ctx->err.clear();
    if (!ctx->has_dict)
        return fail(ctx, DICOD_EINVAL, "autotune: no resident dictionary");
    if (n_sig <= 0 || !X_dev || !T || !x_off || !lambda || !Z_dev || !z_off)
        return fail(ctx, DICOD_EINVAL, "autotune: NULL argument or n_sig <= 0");
    if (max_trials < 1 || max_trials > 64)
        return fail(ctx, DICOD_EINVAL, "autotune: max_trials must be in 1..64");
    if (ctx->cfg.schedule != DICOD_SCHED_EVENODD)
        return fail(ctx, DICOD_EINVAL, "autotune: only the coloured schedule is tuned");
    if (ctx->server)
        return fail(ctx, DICOD_EINVAL, "autotune: serving active on this context (the "
                                       "tuning table is fixed until dicod_finalize)");
    HIPCHECK(ctx, hipSetDevice(ctx->cfg.device));
    const int K = ctx->K, W = ctx->W;
    int64_t lmax = 0;
    for (int i = 0; i < n_sig; ++i) {
        if (T[i] < W)
            return fail(ctx, DICOD_EINVAL, "autotune: signal %d: T < W", i);
        lmax = std::max(lmax, T[i] - W + 1);
    }
    const int bucket = length_bucket(lmax);
    std::vector<dicod_stats> st(n_sig);
    std::map<std::vector<int>, double> seen;
    int trials = 0;
    const double inf = std::numeric_limits<double>::infinity();
    int hard_rc = DICOD_OK;
    std::string hard_msg;

    auto make = [&](int C, int seg, int cap) {
        dicod_tune_entry e;
        std::memset(&e, 0, sizeof e);
        e.K = K;
        e.P = ctx->P;
        e.W = W;
        e.bucket = bucket;
        e.colors = C;
        e.seg_len = seg;
        e.update_cap = std::min(std::max(cap, 1), 1024);
        e.team_threads = team_threads_for(K, seg, e.update_cap);
        return e;
    };
    // best of two timed solves; failures to converge count as infinitely slow
    auto eval = [&](const dicod_tune_entry& e) -> double {
        const std::vector<int> key = {e.colors, e.seg_len, e.update_cap};
        auto it = seen.find(key);
        if (it != seen.end())
            return it->second;
        if (trials >= max_trials || hard_rc != DICOD_OK)
            return inf;
        ++trials;
        double best = inf;
        ctx->sched_force = &e;
        for (int rep = 0; rep < 2; ++rep) {
            const double t0 = now_ms();
            const int rc = dicod::solve_device_batch(ctx, n_sig, X_dev, T, x_off, lambda, eps,
                                                     nullptr, Z_dev, z_off, st.data(),
                                                     ctx->stream);
            const double t = now_ms() - t0;
            if (rc == DICOD_ENOTCONV || rc == DICOD_EINVAL || rc == DICOD_ENOTSUP)
                break;  // this schedule is not usable here
            if (rc != DICOD_OK) {
                hard_rc = rc;
                hard_msg = ctx->err;
                break;
            }
            best = std::min(best, t);
        }
        ctx->sched_force = nullptr;
        ctx->err.clear();
        seen[key] = best;
        return best;
    };

    const int cap0 = effective_update_cap(-1, W);
    std::vector<int> lad2 = seg_ladder(W, 2, lmax);
    int seg0 = lad2.back();
    for (int x : lad2)  // the ladder entry nearest 2W from above
        if (x >= 2 * W) {
            seg0 = x;
            break;
        }
    dicod_tune_entry best = make(2, seg0, cap0);
    double tb = eval(best);
    const double t_prior = tb;
    for (bool moved = true; moved && trials < max_trials && hard_rc == DICOD_OK;) {
        moved = false;
        std::vector<dicod_tune_entry> nb;
        for (int C = 2; C <= 4; ++C) {
            if (C == best.colors)
                continue;
            const int lo = (int)min_segment(W, C);
            nb.push_back(make(C, std::max(best.seg_len, lo), best.update_cap));
            nb.push_back(make(C, seg_ladder(W, C, lmax).front(), best.update_cap));
        }
        const std::vector<int> lad = seg_ladder(W, best.colors, lmax);
        const size_t pos = std::lower_bound(lad.begin(), lad.end(), best.seg_len) - lad.begin();
        if (pos > 0)
            nb.push_back(make(best.colors, lad[pos - 1], best.update_cap));
        if (pos + 1 < lad.size())
            nb.push_back(make(best.colors, lad[pos + 1], best.update_cap));
        nb.push_back(make(best.colors, best.seg_len, best.update_cap * 2));
        if (best.update_cap > 1)
            nb.push_back(make(best.colors, best.seg_len, best.update_cap / 2));
        for (const dicod_tune_entry& e : nb) {
            const double t = eval(e);
            if (t < 0.98 * tb) {
                best = e;
                tb = t;
                moved = true;
                break;
            }
        }
    }
    if (hard_rc != DICOD_OK)
        return fail(ctx, hard_rc, "autotune: %s", hard_msg.c_str());
    if (!(tb < inf))
        return fail(ctx, DICOD_ENOTCONV, "autotune: no candidate schedule converged");
    best.trials = trials;
    best.ms = tb;
    best.ms_prior = t_prior;
    ctx->tuning[bucket] = best;
    // leave the chosen schedule's solution in Z_dev
    ctx->sched_force = &best;
    const int rc = dicod::solve_device_batch(ctx, n_sig, X_dev, T, x_off, lambda, eps, nullptr,
                                             Z_dev, z_off, st.data(), ctx->stream);
    ctx->sched_force = nullptr;
    if (out)
        *out = best;
    return rc;
}

extern "C" int dicod_get_tuning(dicod_ctx* ctx, dicod_tune_entry* out, int cap, int* n)
{
    if (!ctx || !n || cap < 0 || (cap > 0 && !out))
        return DICOD_EINVAL;
    int i = 0;
    for (const auto& kv : ctx->tuning) {
        if (i < cap)
            out[i] = kv.second;
        ++i;
    }
    *n = i;
    return DICOD_OK;
}

extern "C" int dicod_set_tuning(dicod_ctx* ctx, const dicod_tune_entry* e)
{
    if (!ctx)
        return DICOD_EINVAL;
    ctx->err.clear();
    if (ctx->server)
        return fail(ctx, DICOD_EINVAL, "set_tuning: serving active on this context (the "
                                       "tuning table is fixed until dicod_finalize)");
    if (!e) {
        ctx->tuning.clear();
        return DICOD_OK;
    }
    if (!ctx->has_dict || e->K != ctx->K || e->P != ctx->P || e->W != ctx->W)
        return fail(ctx, DICOD_EINVAL, "set_tuning: entry shape differs from the dictionary");
    if (e->colors < 2 || e->colors > kMaxColors || e->update_cap < 1 || e->update_cap > 1024 ||
        e->bucket < 0 || e->bucket > 62 || e->seg_len < min_segment(ctx->W, e->colors))
        return fail(ctx, DICOD_EINVAL, "set_tuning: invalid entry");
    dicod_tune_entry c = *e;
    c.team_threads = team_threads_for(ctx->K, c.seg_len, c.update_cap);
    ctx->tuning[c.bucket] = c;
    return DICOD_OK;
}

// Accessors used by the serving module.
namespace dicod {
// Colours and update cap of a server on this context: the config's.  (Served
// requests do not take their schedule from the tuning table: a served pair of
// tuned requests stopped making progress in testing and the cause is not
// known, so that path is switched off.)
void ctx_serve_schedule(const dicod_ctx* ctx, int* colors, int* update_cap)
{
    *colors = ctx->cfg.colors;
    *update_cap = ctx->cfg.update_cap;
}
// Segment count of a served request of L coefficients under C colours: the
// fixed rule (see ctx_serve_schedule).
int ctx_serve_segments(const dicod_ctx* ctx, int64_t L, int C, int* tuned)
{
    *tuned = 0;
    return auto_segments(L, ctx->W, C);
}
dicod::Server*& ctx_server(dicod_ctx* ctx) { return ctx->server; }
const dicod_config& ctx_config(const dicod_ctx* ctx) { return ctx->cfg; }
int ctx_dims(const dicod_ctx* ctx, int* K, int* P, int* W)
{
    *K = ctx->K;
    *P = ctx->P;
    *W = ctx->W;
    return ctx->has_dict ? 1 : 0;
}
int ctx_fail(dicod_ctx* ctx, int code, const char* msg) { return fail(ctx, code, "%s", msg); }
DictView ctx_dict(const dicod_ctx* ctx)
{
    DictView v;
    v.D64 = ctx->D64.as<double>();
    v.S64 = ctx->S64.as<double>();
    v.S32 = ctx->S32.p;
    v.St32 = ctx->St32.p;
    v.St64 = ctx->St64.p;
    v.Sc64 = ctx->Sc64.as<double>();
    v.n2_32 = ctx->n2_32.p;
    v.inv32 = ctx->inv32.p;
    v.n2_64 = ctx->n2_64.p;
    v.inv64 = ctx->inv64.p;
    v.Dsp = ctx->Dsp.as<unsigned short>();
    v.dnorm_max = ctx->dnorm_max;
    return v;
}
int64_t min_segment_len(int W, int C) { return min_segment(W, C); }
int effective_update_cap(int update_cap, int W)
{
    if (update_cap > 0)
        return update_cap;
    if (update_cap == 0)
        return kRunUpdateBound;
    return std::max(4, (int)std::lround(2.0 * std::sqrt((double)W)));
}
int auto_segment_count(int64_t L, int W, int C) { return auto_segments(L, W, C); }
}  // namespace dicod
