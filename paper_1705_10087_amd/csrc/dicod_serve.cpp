// Serving loop of the LGCD library: continuous batching of encode requests
// against the resident dictionary.
//
// Device arenas are sized from the HBM budget at the first dicod_submit:
// coefficient arenas (Z, beta0, float and double g, all indexed by one
// element offset), a sample arena (X) and a segment table, each handed out by
// a first-fit range allocator.  Requests are served by two lanes, one for
// short requests (few segments) and one for the rest, each a scheduler thread
// with its own HIP stream and phase cadence, so that short requests do not
// wait for the phases of long ones.  A lane admits its requests in arrival
// order while a slot and the three ranges are free (admission by footprint).
// An admitted request is initialised (beta at Z = 0 on double MFMA in every
// precision policy, lambda, Z = 0)
// and joins the coloured phases ("ticks") of the lane's running set: every
// tick launches one phase kernel per state class over the segments of all
// running requests that their own phase counter selects.
// A request counts its phases from its admission, so its sequence of segment
// runs, and hence its result, does not depend on the requests it shares the
// device with.  When C consecutive phases of a request apply no update, that
// request alone is checked in double precision (the stop test of Sec. 2.1)
// and either completes or resumes on a refreshed state, the same sequence of
// rounds as a one-shot solve.  dicod_poll copies a completed Z to the caller
// and returns the request's memory to the allocators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dicod_internal.h"
#include "dicod_serve.h"

namespace dicod {
namespace {

constexpr int kRing = 64;       // phases of per-request update counts kept
constexpr int kMaxChunk = 32;   // phases launched between host polls
constexpr int kLanes = 2;
constexpr int kShortSegs = 256; // requests of at most this many segments: lane 0

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

int64_t round_up(int64_t n, int64_t a) { return (n + a - 1) / a * a; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device allocation owned by the server (allocated once, freed at teardown).
struct Mem {
    void* p = nullptr;
    hipError_t alloc(size_t bytes)
    {
        return hipMalloc(&p, bytes < 256 ? 256 : bytes);
    }
    void release()
    {
        if (p)
            (void)hipFree(p);
        p = nullptr;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// First-fit allocator of ranges of [0, cap), coalescing on release.
class RangeAlloc {
public:
    void reset(int64_t cap)
    {
        cap_ = cap;
        free_.clear();
        if (cap > 0)
            free_[0] = cap;
    }
    bool alloc(int64_t n, int64_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n)
                continue;
            const int64_t o = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n)
                free_[o + n] = sz - n;
            *off = o;
            return true;
        }
        return false;
    }
    void release(int64_t off, int64_t n)
    {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t capacity() const { return cap_; }

private:
    int64_t cap_ = 0;
    std::map<int64_t, int64_t> free_;
};

// Pinned host buffers in power-of-two size classes, reused and released only
// at teardown (freeing pinned memory can wait for the whole device).
class PinnedPool {
public:
    void* get(size_t bytes, size_t* cls)
    {
        size_t c = (size_t)1 << 16;
        while (c < bytes)
            c <<= 1;
        std::lock_guard<std::mutex> g(mu_);
        auto it = free_.find(c);
        if (it != free_.end()) {
            void* p = it->second;
            free_.erase(it);
            *cls = c;
            return p;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess)
            return nullptr;
        all_.push_back(p);
        *cls = c;
        return p;
    }
    void put(void* p, size_t cls)
    {
        if (!p)
            return;
        std::lock_guard<std::mutex> g(mu_);
        free_.emplace(cls, p);
    }
    ~PinnedPool()
    {
        for (void* p : all_)
            (void)hipHostFree(p);
    }

private:
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    std::vector<void*> all_;
};

enum JobState { kQueued, kRunning, kDone, kCopying };

struct Job {
    uint64_t id = 0;
    int state = kQueued;
    float* hx = nullptr;   // pinned copy of X until it is on the device
    size_t hx_cls = 0;
    int64_t T = 0, L = 0;
    int M = 0, lm = 0, lext = 0;
    double lam_in = 0.0, eps = 0.0, lam = 0.0, lmax = 0.0;
    int slot = -1;
    int64_t z_off = 0, zn = 0, x_off = 0, xn = 0, seg_base = 0;
    bool cur64 = false, in_lds = false, lds64 = false, lds32 = false;
    bool reg32 = false;           // float rounds on the register-state kernel
    int tuned = 0;                // segment count from the tuning table
    int lane = 0;
    bool polished = false, any_hbm = false, out_of_phases = false;
    int n_refresh = 0, round = 0;
    int64_t start = 0;            // tick of local phase 0 of the current round
    int64_t phases = 0;           // phases of finished rounds
    unsigned long long upd_round0 = 0, upd = 0;
    int64_t round_upd[4] = {0, 0, 0, 0}, round_ph[4] = {0, 0, 0, 0};
    int round_state[4] = {0, 0, 0, 0};
    double round_mdz[4] = {0.0, 0.0, 0.0, 0.0};
    int rc = DICOD_OK;
    std::string err;
    CheckResult res{};
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
};

}  // namespace

struct Server;

// One scheduling lane: a thread, a stream, its running requests, its phase
// counter and the scratch of its launches and checks.
struct Lane {
    Server* srv = nullptr;
    int id = 0;
    hipStream_t s = nullptr;
    std::thread th;
    std::vector<Job*> running;  // this lane's thread only
    int64_t tick = 0;
    int queued = 0;             // requests of this lane in the queue (mu)
    uint64_t blocked = ~0ull;   // epoch at which admission last found no room (mu)
    std::string msg;            // last HIP failure
    Mem dRing, dLists, dSub, dTilesL, dTilesC, dTilesA, dTilesN, dPart, dRes, dLmax,
        dDone, dSlots, dLamIn, dMask;
    // MIXED policy: the double beta0 of admitted requests runs on a side
    // stream beside the descent; ev_b marks the last one queued
    hipStream_t side = nullptr;
    hipEvent_t ev_x = nullptr, ev_b = nullptr;
    bool beta_pending = false;
    Mem dEbits, dThr;
    unsigned long long* h_ring = nullptr;
    unsigned long long* h_sigupd = nullptr;
    unsigned long long* h_lmax = nullptr;
    CheckResult* h_res = nullptr;
    unsigned char* h_stage = nullptr;
    size_t stage_cap = 0, stage_off = 0;

    int start();
    void teardown();
    void loop();
    int iterate(int* admitted);
    void admit(std::vector<Job*>& fresh);
    int init_jobs(const std::vector<Job*>& fresh);
    int check_jobs(const std::vector<Job*>& conv, std::vector<Job*>& resumed);
    void abandon(int rc, const std::string& m);
    hipError_t stage(void* dst, const void* src, size_t bytes);
};

struct Server {
    dicod_ctx* ctx = nullptr;
    dicod_config cfg{};
    int K = 0, P = 0, W = 0, C = 2;
    bool fp64 = false;
    bool mixed = false;          // split-bf16 float start (MIXED policy)
    DictView dict{};
    hipStream_t cs = nullptr;    // result copies (dicod_poll)
    std::mutex mu;               // queue, jobs, allocators, slots, lane counters
    std::mutex copy_mu;          // the copy stream
    std::condition_variable cv;
    bool stop = false;
    uint64_t epoch = 0;          // bumped by every submit and release
    int fatal = DICOD_OK;
    std::string fatal_msg;
    std::deque<Job*> queue;
    std::unordered_map<uint64_t, Job*> jobs;
    uint64_t next_id = 1;
    std::vector<int> free_slots;
    RangeAlloc coef, samp, segr;
    int slots = 0;
    int64_t seg_cap = 0, tilesC_cap = 0, mask_cap = 0;
    int chunk = 16;
    // shared device state, indexed by ranges and slots
    Mem dX, dZ, dB, dG32, dG64, dSig, dSeg, dDirty, dSigUpd, dSigLast, dCnt;
    Mem dBox, dBoxN, dZ32;       // register kernel: mailboxes, float copy of Z
    int box_cap = 0;
    SigDesc* h_sig = nullptr;    // host mirror, one entry per slot
    PinnedPool pool;
    Lane lanes[kLanes];

    ~Server();
    int start(dicod_ctx* c);
    void finish(Job* j, int rc, const char* msg);
    void release(Job* j);
    void fail_all(int rc, const std::string& msg);
};

#define SRV_HIP(expr)                                                                  \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess) {                                                        \
            msg = std::string(#expr) + ": " + hipGetErrorString(_e);                   \
            return _e == hipErrorOutOfMemory ? DICOD_ENOMEM : DICOD_EDEVICE;           \
        }                                                                              \
    } while (0)

hipError_t Lane::stage(void* dst, const void* src, size_t bytes)
{
    if (bytes == 0)
        return hipSuccess;
    const size_t off = (stage_off + 255) & ~(size_t)255;
    if (off + bytes > stage_cap)
        return hipErrorOutOfMemory;
    std::memcpy(h_stage + off, src, bytes);
    stage_off = off + bytes;
    return hipMemcpyAsync(dst, h_stage + off, bytes, hipMemcpyHostToDevice, s);
}

int Lane::start()
{
    const int slots = srv->slots;
    const int n_kblk = check_kblocks(srv->K, srv->W);
    SRV_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    SRV_HIP(dRing.alloc((size_t)slots * kRing * sizeof(unsigned long long)));
    SRV_HIP(dLists.alloc((size_t)srv->seg_cap * sizeof(int32_t)));
    SRV_HIP(dSub.alloc((size_t)slots * sizeof(SigDesc)));
    SRV_HIP(dTilesL.alloc((size_t)(slots + 1) * sizeof(int64_t)));
    SRV_HIP(dTilesC.alloc((size_t)(slots + 1) * sizeof(int64_t)));
    SRV_HIP(dTilesA.alloc((size_t)(slots + 1) * sizeof(int64_t)));
    SRV_HIP(dTilesN.alloc((size_t)(slots + 1) * sizeof(int64_t)));
    SRV_HIP(dMask.alloc((size_t)srv->mask_cap * sizeof(unsigned long long)));
    SRV_HIP(dPart.alloc((size_t)srv->tilesC_cap * n_kblk * kCheckParts * sizeof(double)));
    SRV_HIP(dRes.alloc((size_t)slots * sizeof(CheckResult)));
    SRV_HIP(dLmax.alloc((size_t)slots * sizeof(unsigned long long)));
    SRV_HIP(dDone.alloc((size_t)slots * sizeof(uint32_t)));
    SRV_HIP(dSlots.alloc((size_t)slots * sizeof(int)));
    SRV_HIP(dLamIn.alloc((size_t)slots * sizeof(double)));
    SRV_HIP(launch_fill_u32(dDone.as<uint32_t>(), 0u, slots, s));
    if (srv->mixed) {
        SRV_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        SRV_HIP(hipEventCreateWithFlags(&ev_x, hipEventDisableTiming));
        SRV_HIP(hipEventCreateWithFlags(&ev_b, hipEventDisableTiming));
        SRV_HIP(dEbits.alloc((size_t)slots * sizeof(unsigned long long)));
        SRV_HIP(dThr.alloc((size_t)slots * sizeof(double)));
    }
    stage_cap = (size_t)srv->seg_cap * sizeof(int32_t) +
                2 * (size_t)srv->seg_cap * sizeof(SegDesc) +
                8 * (size_t)(slots + 1) * (sizeof(SigDesc) + 3 * sizeof(int64_t) + 16) +
                ((size_t)1 << 20);
    SRV_HIP(hipHostMalloc((void**)&h_stage, stage_cap, hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&h_ring, (size_t)slots * kRing * sizeof(unsigned long long),
                          hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&h_sigupd, (size_t)slots * sizeof(unsigned long long),
                          hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&h_lmax, (size_t)slots * sizeof(unsigned long long),
                          hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&h_res, (size_t)slots * sizeof(CheckResult),
                          hipHostMallocDefault));
    SRV_HIP(hipStreamSynchronize(s));
    th = std::thread([this] { loop(); });
    return DICOD_OK;
}

void Lane::teardown()
{
    if (th.joinable())
        th.join();
    if (s)
        (void)hipStreamSynchronize(s);
    if (side)
        (void)hipStreamSynchronize(side);
    for (Mem* m : {&dRing, &dLists, &dSub, &dTilesL, &dTilesC, &dTilesA, &dTilesN, &dPart,
                   &dRes, &dLmax, &dDone, &dSlots, &dLamIn, &dMask, &dEbits, &dThr})
        m->release();
    for (hipEvent_t* e : {&ev_x, &ev_b})
        if (*e) {
            (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    if (side)
        (void)hipStreamDestroy(side);
    side = nullptr;
    for (void* p : {(void*)h_stage, (void*)h_ring, (void*)h_sigupd, (void*)h_lmax,
                    (void*)h_res})
        if (p)
            (void)hipHostFree(p);
    if (s)
        (void)hipStreamDestroy(s);
    s = nullptr;
}

int Server::start(dicod_ctx* c)
{
    std::string& msg = fatal_msg;
    ctx = c;
    cfg = ctx_config(c);
    ctx_dims(c, &K, &P, &W);
    ctx_serve_schedule(c, &cfg.colors, &cfg.update_cap);
    C = cfg.colors;
    fp64 = cfg.precision == DICOD_PREC_FP64;
    mixed = cfg.precision == DICOD_PREC_MIXED;
    dict = ctx_dict(c);
    slots = cfg.max_inflight;
    chunk = std::min(std::max(cfg.phases_per_poll, 1), kMaxChunk);
    SRV_HIP(hipSetDevice(cfg.device));
    SRV_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    size_t budget = cfg.hbm_budget_bytes;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        SRV_HIP(hipMemGetInfo(&fr, &tot));
        budget = std::min<size_t>((size_t)(0.8 * (double)fr), (size_t)16 << 30);
    }
    // bytes per coefficient: Z, beta0 and the double g; the float g and the
    // float copy of Z in FP32
    // (the lanes' non-zero masks, 1/8 byte per coefficient each, fit in the
    // 5% left over)
    const int64_t bc = fp64 ? 24 : 32;
    const int64_t bs = 4;
    const double share = (double)(bc * K) / (double)(bc * K + bs * P);
    const int64_t n_coef = round_up((int64_t)(share * 0.95 * (double)budget) / bc, 64);
    const int64_t n_samp = round_up((int64_t)((1.0 - share) * 0.95 * (double)budget) / bs, 64);
    if (n_coef <= 0 || n_samp <= 0) {
        msg = "hbm_budget_bytes too small";
        return DICOD_ENOMEM;
    }
    coef.reset(n_coef);
    samp.reset(n_samp);
    seg_cap = n_coef / ((int64_t)K * min_segment_len(W, C)) + slots + 16;
    segr.reset(seg_cap);
    tilesC_cap = n_coef / K / kCheckSpan + slots + 1;
    // each request rounds every atom row up to whole 64-bit words
    mask_cap = n_coef / 64 + (int64_t)slots * K + 1;
    SRV_HIP(dX.alloc((size_t)n_samp * sizeof(float)));
    SRV_HIP(dZ.alloc((size_t)n_coef * sizeof(double)));
    SRV_HIP(dB.alloc((size_t)n_coef * sizeof(double)));
    SRV_HIP(dG64.alloc((size_t)n_coef * sizeof(double)));
    if (!fp64) {
        SRV_HIP(dG32.alloc((size_t)n_coef * sizeof(float)));
        SRV_HIP(dZ32.alloc((size_t)n_coef * sizeof(float)));
        box_cap = std::max(effective_update_cap(cfg.update_cap, W), 1);
        SRV_HIP(dBox.alloc((size_t)2 * seg_cap * box_cap * sizeof(BoundaryRec)));
        SRV_HIP(dBoxN.alloc((size_t)2 * seg_cap * sizeof(uint32_t)));
    }
    SRV_HIP(dSig.alloc((size_t)slots * sizeof(SigDesc)));
    SRV_HIP(dSeg.alloc((size_t)seg_cap * sizeof(SegDesc)));
    SRV_HIP(dDirty.alloc((size_t)seg_cap * sizeof(uint32_t)));
    SRV_HIP(dSigUpd.alloc((size_t)slots * sizeof(unsigned long long)));
    SRV_HIP(dSigLast.alloc((size_t)slots * sizeof(int)));
    SRV_HIP(dCnt.alloc(sizeof(Counters)));
    SRV_HIP(launch_fill_u64(dCnt.as<unsigned long long>(), 0ull, sizeof(Counters) / 8, cs));
    SRV_HIP(hipHostMalloc((void**)&h_sig, (size_t)slots * sizeof(SigDesc), hipHostMallocDefault));
    SRV_HIP(hipStreamSynchronize(cs));
    for (int i = slots - 1; i >= 0; --i)
        free_slots.push_back(i);
    for (int l = 0; l < kLanes; ++l) {
        lanes[l].srv = this;
        lanes[l].id = l;
        const int rc = lanes[l].start();
        if (rc != DICOD_OK) {
            msg = lanes[l].msg;
            return rc;
        }
    }
    return DICOD_OK;
}

Server::~Server()
{
    {
        std::lock_guard<std::mutex> g(mu);
        stop = true;
    }
    cv.notify_all();
    for (Lane& l : lanes)
        l.teardown();
    (void)hipSetDevice(cfg.device);
    if (cs)
        (void)hipStreamSynchronize(cs);
    for (auto& kv : jobs) {
        pool.put(kv.second->hx, kv.second->hx_cls);
        delete kv.second;
    }
    for (Mem* m : {&dX, &dZ, &dB, &dG32, &dG64, &dSig, &dSeg, &dDirty, &dSigUpd, &dSigLast,
                   &dCnt, &dBox, &dBoxN, &dZ32})
        m->release();
    if (h_sig)
        (void)hipHostFree(h_sig);
    if (cs)
        (void)hipStreamDestroy(cs);
}

// Completion of a request (lane thread, mu not held).
void Server::finish(Job* j, int rc, const char* m)
{
    j->rc = rc;
    if (m)
        j->err = m;
    j->t_done = now_ms();
    std::lock_guard<std::mutex> g(mu);
    j->state = kDone;
}

// Returns a request's device ranges and slot (mu held).
void Server::release(Job* j)
{
    if (j->slot >= 0) {
        coef.release(j->z_off, j->zn);
        samp.release(j->x_off, j->xn);
        segr.release(j->seg_base, j->M);
        free_slots.push_back(j->slot);
        j->slot = -1;
    }
}

// A HIP failure in a lane ends serving: every open request fails with it
// (mu not held).
void Server::fail_all(int rc, const std::string& m)
{
    {
        std::lock_guard<std::mutex> g(mu);
        if (fatal == DICOD_OK) {  // the first failure names the cause
            fatal = rc;
            fatal_msg = m;
        }
        stop = true;
        // queued requests belong to no lane; running ones are failed by their
        // lane once it has stopped using them (Lane::abandon)
        for (Job* j : queue) {
            j->rc = rc;
            j->err = m;
            j->state = kDone;
            j->t_done = now_ms();
        }
        queue.clear();
        for (Lane& l : lanes)
            l.queued = 0;
    }
    cv.notify_all();
}

void Lane::loop()
{
    if (hipSetDevice(srv->cfg.device) != hipSuccess) {
        srv->fail_all(DICOD_EDEVICE, "serving thread: hipSetDevice failed");
        return;
    }
    for (;;) {
        uint64_t seen;
        {
            std::unique_lock<std::mutex> g(srv->mu);
            srv->cv.wait(g, [this] {
                return srv->stop || !running.empty() ||
                       (queued > 0 && !srv->free_slots.empty() && srv->epoch != blocked);
            });
            if (srv->stop) {
                const int frc = srv->fatal;
                const std::string fm = srv->fatal_msg;
                g.unlock();
                abandon(frc, fm);
                return;
            }
            seen = srv->epoch;
        }
        int admitted = 0;
        const int rc = iterate(&admitted);
        if (rc != DICOD_OK) {
            const std::string m = "serving: " + msg;
            srv->fail_all(rc, m);
            abandon(rc, m);
            return;
        }
        if (running.empty() && admitted == 0) {
            // the lane's next request waits for memory held by other requests
            std::lock_guard<std::mutex> g(srv->mu);
            blocked = seen;
        }
    }
}

// The lane stops: its running requests fail with rc when serving failed
// (rc != DICOD_OK; at teardown they are simply dropped with the server).
void Lane::abandon(int rc, const std::string& m)
{
    if (side)  // no double beta0 left writing into ranges about to be freed
        (void)hipStreamSynchronize(side);
    if (rc != DICOD_OK) {
        const double t = now_ms();
        std::lock_guard<std::mutex> g(srv->mu);
        for (Job* j : running) {
            j->rc = rc;
            j->err = m;
            j->t_done = t;
            j->state = kDone;
        }
    }
    running.clear();
    srv->cv.notify_all();
}

// Admission of this lane's requests in arrival order while a slot and the
// three ranges are free.
void Lane::admit(std::vector<Job*>& fresh)
{
    std::lock_guard<std::mutex> g(srv->mu);
    for (auto it = srv->queue.begin(); it != srv->queue.end() && !srv->free_slots.empty();) {
        Job* j = *it;
        if (j->lane != id) {
            ++it;
            continue;
        }
        int64_t zo, xo, so;
        if (!srv->coef.alloc(j->zn, &zo))
            break;
        if (!srv->samp.alloc(j->xn, &xo)) {
            srv->coef.release(zo, j->zn);
            break;
        }
        if (!srv->segr.alloc(j->M, &so)) {
            srv->coef.release(zo, j->zn);
            srv->samp.release(xo, j->xn);
            break;
        }
        it = srv->queue.erase(it);
        --queued;
        j->z_off = zo;
        j->x_off = xo;
        j->seg_base = so;
        j->slot = srv->free_slots.back();
        srv->free_slots.pop_back();
        j->state = kRunning;
        j->t_admit = now_ms();
        fresh.push_back(j);
    }
}

// beta0 and g on MFMA, lambda on the device, Z = 0, every segment dirty.
// MIXED: g starts from the split-bf16 correlation, lambda_max is made exact
// by the double recomputation of every entry the split's error bound could
// make the maximum (as in the one-shot solver), and the double beta0, read
// only by the requests' first check, runs on the side stream.
int Lane::init_jobs(const std::vector<Job*>& fresh)
{
    Server& v = *srv;
    const int K = v.K, P = v.P, W = v.W;
    const int n = (int)fresh.size();
    // the descriptors staged below are read by the previous side-stream
    // correlation until it ends
    if (beta_pending)
        SRV_HIP(hipStreamWaitEvent(s, ev_b, 0));
    std::vector<SigDesc> sub(n);
    std::vector<int64_t> pL(n + 1, 0), pA(n + 1, 0);
    std::vector<int> sl(n);
    std::vector<double> lin(n);
    for (int i = 0; i < n; ++i) {
        Job* j = fresh[i];
        SigDesc& d = v.h_sig[j->slot];
        d.x_off = j->x_off;
        d.z_off = j->z_off;
        d.T = j->T;
        d.L = j->L;
        d.seg_base = (int32_t)j->seg_base;
        d.M = j->M;
        d.lam = 0.0;  // set on the device below
        d.eps_stop = v.fp64 ? j->eps : j->eps * v.cfg.inner_eps_factor;
        sub[i] = d;
        sl[i] = j->slot;
        lin[i] = j->lam_in;
        pL[i + 1] = pL[i] + ceil_div(j->L, kTile);
        pA[i + 1] = pA[i] + ceil_div((int64_t)K * j->L, kAbsChunk);
        std::vector<SegDesc> segs(j->M);
        for (int m = 0; m < j->M; ++m) {
            SegDesc& e = segs[m];
            e.z_off = j->z_off;
            e.L = (int32_t)j->L;
            e.b = (int32_t)(((__int128)m * j->L) / j->M);
            e.e = (int32_t)(((__int128)(m + 1) * j->L) / j->M);
            e.sig = j->slot;
            e.left = m > 0 ? (int32_t)(j->seg_base + m - 1) : -1;
            e.right = m < j->M - 1 ? (int32_t)(j->seg_base + m + 1) : -1;
        }
        SRV_HIP(stage(v.dSeg.as<SegDesc>() + j->seg_base, segs.data(),
                      segs.size() * sizeof(SegDesc)));
        SRV_HIP(stage(v.dSig.as<SigDesc>() + j->slot, &d, sizeof(SigDesc)));
        SRV_HIP(hipMemcpyAsync(v.dX.as<float>() + j->x_off, j->hx,
                               (size_t)P * j->T * sizeof(float), hipMemcpyHostToDevice, s));
    }
    SRV_HIP(stage(dSub.p, sub.data(), n * sizeof(SigDesc)));
    SRV_HIP(stage(dTilesL.p, pL.data(), (n + 1) * sizeof(int64_t)));
    SRV_HIP(stage(dTilesA.p, pA.data(), (n + 1) * sizeof(int64_t)));
    SRV_HIP(stage(dSlots.p, sl.data(), n * sizeof(int)));
    SRV_HIP(stage(dLamIn.p, lin.data(), n * sizeof(double)));
    if (v.mixed) {
        const float* dX = v.dX.as<float>();
        unsigned long long* lmax = dLmax.as<unsigned long long>();
        SRV_HIP(launch_corr_bf16x3(v.dict.Dsp, K, P, W, dX, dSub.as<SigDesc>(),
                                   dTilesL.as<int64_t>(), n, pL[n], v.dG32.as<float>(), s));
        SRV_HIP(launch_fill_u64(lmax, 0ull, n, s));
        SRV_HIP(launch_fill_u64(dEbits.as<unsigned long long>(), 0ull, n, s));
        SRV_HIP(launch_absmax_f32(v.dG32.as<float>(), K, dSub.as<SigDesc>(),
                                  dTilesA.as<int64_t>(), n, pA[n], lmax, s));
        SRV_HIP(launch_win_energy_max(dX, P, W, dSub.as<SigDesc>(), dTilesL.as<int64_t>(), n,
                                      pL[n], dEbits.as<unsigned long long>(), s));
        SRV_HIP(launch_refine_threshold(lmax, dEbits.as<unsigned long long>(), n,
                                        refine_coef(P, W, v.dict.dnorm_max), dThr.as<double>(),
                                        s));
        SRV_HIP(launch_fill_u64(lmax, 0ull, n, s));
        SRV_HIP(launch_refine_absmax(v.dG32.as<float>(), v.dict.D64, dX, K, P, W,
                                     dSub.as<SigDesc>(), dTilesA.as<int64_t>(), n, pA[n],
                                     dThr.as<double>(), lmax, s));
        SRV_HIP(hipEventRecord(ev_x, s));
        SRV_HIP(hipStreamWaitEvent(side, ev_x, 0));
        SRV_HIP(launch_corr_f64_x32(v.dict.D64, K, P, W, dX, dSub.as<SigDesc>(),
                                    dTilesL.as<int64_t>(), n, pL[n], v.dB.as<double>(), nullptr,
                                    nullptr, side));
        SRV_HIP(hipEventRecord(ev_b, side));
        beta_pending = true;
    } else {
        SRV_HIP(launch_corr_f64_x32(v.dict.D64, K, P, W, v.dX.as<float>(), dSub.as<SigDesc>(),
                                    dTilesL.as<int64_t>(), n, pL[n], v.dB.as<double>(),
                                    v.fp64 ? nullptr : v.dG32.as<float>(),
                                    v.fp64 ? v.dG64.as<double>() : nullptr, s));
        SRV_HIP(launch_fill_u64(dLmax.as<unsigned long long>(), 0ull, n, s));
        SRV_HIP(launch_absmax(v.dB.as<double>(), K, dSub.as<SigDesc>(),
                              dTilesA.as<int64_t>(), n, pA[n], dLmax.as<unsigned long long>(),
                              s));
    }
    SRV_HIP(launch_apply_lambda(v.dSig.as<SigDesc>(), dSlots.as<int>(), dLamIn.as<double>(),
                                dLmax.as<unsigned long long>(), n, s));
    SRV_HIP(hipMemcpyAsync(h_lmax, dLmax.p, n * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    for (Job* j : fresh) {
        SRV_HIP(launch_fill_f64(v.dZ.as<double>() + j->z_off, 0.0, (size_t)K * j->L, s));
        SRV_HIP(launch_fill_u32(v.dDirty.as<uint32_t>() + j->seg_base, 1u, j->M, s));
        if (!v.fp64) {
            SRV_HIP(launch_fill_u32(v.dZ32.as<uint32_t>() + j->z_off, 0u, (size_t)K * j->L, s));
            SRV_HIP(launch_fill_u32(v.dBoxN.as<uint32_t>() + 2 * j->seg_base, 0u,
                                    (size_t)2 * j->M, s));
        }
        SRV_HIP(launch_fill_u64(v.dSigUpd.as<unsigned long long>() + j->slot, 0ull, 1, s));
        j->start = tick;
        j->cur64 = v.fp64;
        j->in_lds = v.fp64 ? j->lds64 : j->lds32;
        j->any_hbm = !j->in_lds && (v.fp64 || !j->reg32);
    }
    return DICOD_OK;
}

// Double-precision stop test of the requests in conv (grouped by state and
// eps), and the decision per request: complete, or refresh and resume at
// colour 0 -- the round structure of the one-shot solver.  The resumed
// requests are appended to `resumed`.  Completed requests are published
// (Server::finish) only after the last access to them here: from then on
// dicod_poll may copy their result and free them at any moment.
int Lane::check_jobs(const std::vector<Job*>& conv, std::vector<Job*>& resumed)
{
    Server& v = *srv;
    const int K = v.K, P = v.P, W = v.W;
    const int n_kblk = check_kblocks(K, W);
    const dicod_config& cfg = v.cfg;
    struct Done {
        Job* j;
        int rc;
        const char* m;
    };
    std::vector<Done> finished;
    if (beta_pending)  // beta0 of the requests admitted under MIXED
        SRV_HIP(hipStreamWaitEvent(s, ev_b, 0));
    // state class of every request (bit 0: double now, bit 1: double in the
    // next round), decided before any request changes state
    std::vector<int> cls(conv.size());
    for (size_t i = 0; i < conv.size(); ++i) {
        const Job* j = conv[i];
        const bool n64 = j->cur64 || (cfg.fp64_polish_after > 0 &&
                                      j->n_refresh + 1 >= cfg.fp64_polish_after);
        cls[i] = (j->cur64 ? 1 : 0) | (n64 ? 2 : 0);
    }
    auto run = [&]() -> int {
        for (int grp = 0; grp < 4; ++grp) {
            const bool c64 = (grp & 1) != 0;
            const bool next64 = (grp & 2) != 0;
            std::vector<Job*> g;
            for (size_t i = 0; i < conv.size(); ++i)
                if (cls[i] == grp)
                    g.push_back(conv[i]);
            if (g.empty())
                continue;
            std::sort(g.begin(), g.end(),
                      [](const Job* a, const Job* b) { return a->eps < b->eps; });
            size_t i0 = 0;
            while (i0 < g.size()) {
                size_t i1 = i0;
                while (i1 < g.size() && g[i1]->eps == g[i0]->eps)
                    ++i1;
                const int n = (int)(i1 - i0);
                const double eps = g[i0]->eps;
                std::vector<SigDesc> sub(n);
                std::vector<int64_t> pC(n + 1, 0), pN(n + 1, 0);
                for (int i = 0; i < n; ++i) {
                    Job* j = g[i0 + i];
                    sub[i] = v.h_sig[j->slot];
                    sub[i].nz_off = pN[i];
                    pC[i + 1] = pC[i] + ceil_div(j->L, kCheckSpan);
                    pN[i + 1] = pN[i] + (int64_t)K * ceil_div(j->L, 64);
                }
                if (pN[n] > v.mask_cap) {
                    msg = "non-zero mask buffer too small";
                    return DICOD_EDEVICE;
                }
                stage_off = 0;  // the previous group was synchronised
                SRV_HIP(stage(dSub.p, sub.data(), n * sizeof(SigDesc)));
                SRV_HIP(stage(dTilesC.p, pC.data(), (n + 1) * sizeof(int64_t)));
                SRV_HIP(stage(dTilesN.p, pN.data(), (n + 1) * sizeof(int64_t)));
                const double flag_eps = next64 ? eps : eps * cfg.inner_eps_factor;
                void* g_next = next64 ? v.dG64.p : v.dG32.p;
                const double* g_in =
                    (c64 && !cfg.verify_from_scratch) ? v.dG64.as<double>() : nullptr;
                if (!g_in)
                    SRV_HIP(launch_nz_mask(v.dZ.as<double>(), dSub.as<SigDesc>(),
                                           dTilesN.as<int64_t>(), n, K, pN[n],
                                           dMask.as<unsigned long long>(), s));
                SRV_HIP(launch_grad_check(v.dX.as<float>(), v.dB.as<double>(),
                                          v.dZ.as<double>(), dMask.as<unsigned long long>(),
                                          v.dict.Sc64, (const double*)v.dict.n2_64, K, P, W,
                                          dSub.as<SigDesc>(), dTilesC.as<int64_t>(), n, pC[n],
                                          flag_eps, dDone.as<uint32_t>(),
                                          v.dDirty.as<uint32_t>(), g_in ? nullptr : g_next,
                                          next64, g_in, dPart.as<double>(),
                                          !next64 && !g_in ? v.dZ32.as<float>() : nullptr,
                                          nullptr, s));
                SRV_HIP(launch_check_reduce(dPart.as<double>(), dTilesC.as<int64_t>(), pC[n],
                                            n_kblk, n, dRes.as<CheckResult>(), s));
                SRV_HIP(hipMemcpyAsync(h_res, dRes.p, n * sizeof(CheckResult),
                                       hipMemcpyDeviceToHost, s));
                std::vector<Job*> res_grp;
                SRV_HIP(hipStreamSynchronize(s));
                for (int i = 0; i < n; ++i) {
                    Job* j = g[i0 + i];
                    j->res = h_res[i];
                    if (j->round >= 1 && j->round <= 4)
                        j->round_mdz[j->round - 1] = j->res.max_dz;
                    const bool ok = j->res.max_dz < j->eps;
                    if (ok || j->out_of_phases || j->n_refresh >= cfg.max_refresh) {
                        finished.push_back(
                            {j, ok ? DICOD_OK : DICOD_ENOTCONV,
                             ok ? nullptr
                                : (j->out_of_phases
                                       ? "max_phases reached before the stop test held"
                                       : "max_refresh double-precision checks failed")});
                        continue;
                    }
                    ++j->n_refresh;
                    if (next64 && !j->cur64) {
                        j->cur64 = true;
                        j->in_lds = j->lds64;
                        j->polished = true;
                        j->any_hbm |= !j->in_lds;
                    }
                    SigDesc& d = v.h_sig[j->slot];
                    d.eps_stop = j->cur64 ? j->eps : j->eps * cfg.inner_eps_factor;
                    res_grp.push_back(j);
                    // the next round starts with colour 0 on the next tick
                    j->start = tick;
                    j->upd_round0 = j->upd;
                }
                stage_off = 0;
                for (Job* j : res_grp) {
                    SRV_HIP(stage(v.dSig.as<SigDesc>() + j->slot, &v.h_sig[j->slot],
                                  sizeof(SigDesc)));
                    if (!v.fp64)  // records of the last round are stale: g was refreshed
                        SRV_HIP(launch_fill_u32(v.dBoxN.as<uint32_t>() + 2 * j->seg_base, 0u,
                                                (size_t)2 * j->M, s));
                }
                SRV_HIP(hipStreamSynchronize(s));
                resumed.insert(resumed.end(), res_grp.begin(), res_grp.end());
                i0 = i1;
            }
        }
        return DICOD_OK;
    };
    const int rc = run();
    if (rc != DICOD_OK) {
        // the lane stops; the requests not yet decided stay in its care and
        // fail with the lane (Lane::abandon)
        for (Job* j : conv) {
            bool decided = false;
            for (const Done& d : finished)
                decided |= d.j == j;
            if (!decided && std::find(resumed.begin(), resumed.end(), j) == resumed.end())
                resumed.push_back(j);
        }
    }
    for (const Done& d : finished)
        v.finish(d.j, d.rc, d.m);
    return rc;
}

// One scheduling step: admission, one chunk of ticks, convergence and checks.
int Lane::iterate(int* admitted)
{
    Server& v = *srv;
    const int K = v.K, W = v.W, C = v.C;
    const dicod_config& cfg = v.cfg;
    stage_off = 0;
    std::vector<Job*> fresh;
    admit(fresh);
    *admitted = (int)fresh.size();
    if (!fresh.empty()) {
        int rc = init_jobs(fresh);
        if (rc != DICOD_OK)
            return rc;
        for (Job* j : fresh)
            running.push_back(j);
    }
    if (running.empty())
        return DICOD_OK;

    // chunk length: no request crosses its round or watchdog limit inside it
    int64_t n = v.chunk;
    for (Job* j : running) {
        const int64_t lp = tick - j->start;
        if (!j->cur64)
            n = std::min<int64_t>(n, kRoundPhaseLimit - lp);
        n = std::min<int64_t>(n, cfg.max_phases - (j->phases + lp));
    }
    n = std::max<int64_t>(n, 1);

    // launch groups: one state class each, small enough that the largest
    // segment of the group fits the kernel's LDS layout; lists per tick
    // residue r = t % C (a request's colour at tick t is (t - start) % C)
    struct Group {
        bool c64, lds, reg;
        int lm, lx;
        std::vector<int32_t> list[kMaxColors];
        size_t off[kMaxColors];
    };
    std::vector<Group> groups;
    for (Job* j : running) {
        Group* gp = nullptr;
        const bool reg = !j->cur64 && j->reg32;
        for (Group& g : groups) {
            if (g.c64 != j->cur64 || g.reg != reg || (!reg && g.lds != j->in_lds))
                continue;
            const int lm = std::max(g.lm, j->lm), lx = std::max(g.lx, j->lext);
            const size_t b = reg ? 0
                           : g.lds ? lgcd_lds_bytes(K, lm, lx, g.c64)
                                   : lgcd_gm_lds_bytes(K, lx, g.c64);
            if (b <= kLdsBytes) {
                gp = &g;
                break;
            }
        }
        if (!gp) {
            groups.emplace_back();
            gp = &groups.back();
            gp->c64 = j->cur64;
            gp->lds = j->in_lds;
            gp->reg = reg;
            gp->lm = 0;
            gp->lx = 0;
        }
        gp->lm = std::max(gp->lm, j->lm);
        gp->lx = std::max(gp->lx, j->lext);
        for (int r = 0; r < C; ++r) {
            const int col = (int)(((r - j->start) % C + C) % C);
            for (int m = col; m < j->M; m += C)
                gp->list[r].push_back((int32_t)(j->seg_base + m));
        }
    }
    size_t loff = 0;
    for (Group& g : groups)
        for (int r = 0; r < C; ++r) {
            g.off[r] = loff;
            SRV_HIP(stage(dLists.as<int32_t>() + loff, g.list[r].data(),
                          g.list[r].size() * sizeof(int32_t)));
            loff += g.list[r].size();
        }
    SRV_HIP(launch_clear_ring(dRing.as<unsigned long long>(), v.slots, kRing,
                              (int)(tick % kRing), (int)n, s));
    PhaseArgs a;
    std::memset(&a, 0, sizeof a);
    a.segs = v.dSeg.as<SegDesc>();
    a.Z = v.dZ.as<double>();
    a.sigs = v.dSig.as<SigDesc>();
    a.K = K;
    a.W = W;
    a.cap = effective_update_cap(cfg.update_cap, W);
    a.phase_stride = kRing;
    a.dirty = v.dDirty.as<uint32_t>();
    a.phase_upd = dRing.as<unsigned long long>();
    a.sig_upd = v.dSigUpd.as<unsigned long long>();
    a.sig_last_upd = v.dSigLast.as<int>();
    a.counters = v.dCnt.as<Counters>();
    a.box = v.fp64 ? nullptr : v.dBox.as<BoundaryRec>();
    a.box_n = v.fp64 ? nullptr : v.dBoxN.as<uint32_t>();
    a.box_cap = v.box_cap;
    a.z32 = v.fp64 ? nullptr : v.dZ32.as<float>();
    for (int64_t t = tick; t < tick + n; ++t) {
        const int r = (int)(t % C);
        for (const Group& g : groups) {
            const size_t nl = g.list[r].size();
            if (nl == 0)
                continue;
            a.list = dLists.as<int32_t>() + g.off[r];
            a.n_list = (int)nl;
            a.phase = (int)(t % kRing);
            a.g = g.c64 ? v.dG64.p : v.dG32.p;
            a.S = g.c64 ? (g.lds ? v.dict.St64 : (const void*)v.dict.S64)
                        : (g.lds ? v.dict.St32 : v.dict.S32);
            a.n2 = g.c64 ? v.dict.n2_64 : v.dict.n2_32;
            a.inv_n2 = g.c64 ? v.dict.inv64 : v.dict.inv32;
            a.lm_max = g.lm;
            a.lext_max = g.lx;
            size_t lds_b = 0;
            hipError_t e = g.reg   ? launch_lgcd_wave(a, s)
                           : g.lds ? launch_lgcd_phase(a, g.c64, &lds_b, s)
                                   : launch_lgcd_phase_gm(a, g.c64, &lds_b, s);
            if (e != hipSuccess) {
                msg = std::string("phase launch: ") + hipGetErrorString(e);
                return DICOD_EDEVICE;
            }
        }
    }
    SRV_HIP(hipMemcpyAsync(h_ring, dRing.p, (size_t)v.slots * kRing * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    SRV_HIP(hipMemcpyAsync(h_sigupd, v.dSigUpd.p, (size_t)v.slots * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    SRV_HIP(hipStreamSynchronize(s));
    const int64_t t0 = tick;
    tick += n;

    // lambda of the requests admitted in this step (the same double product
    // as on the device); their pinned X goes back to the pool
    for (size_t i = 0; i < fresh.size(); ++i) {
        Job* j = fresh[i];
        double lmax;
        std::memcpy(&lmax, &h_lmax[i], sizeof lmax);
        j->lmax = lmax;
        double lam = j->lam_in;
        if (lam < 0.0) {
            lam = -lam * lmax;
            if (!(lam > 0.0))
                lam = 1e-300;
        }
        j->lam = lam;
        v.h_sig[j->slot].lam = lam;
        v.pool.put(j->hx, j->hx_cls);
        j->hx = nullptr;
    }

    // convergence: C consecutive phases of the request without an update
    std::vector<Job*> conv, keep;
    for (Job* j : running) {
        j->upd = h_sigupd[j->slot];
        const unsigned long long* row = h_ring + (size_t)j->slot * kRing;
        int64_t conv_t = -1;
        for (int64_t t = std::max<int64_t>(j->start + C - 1, t0); t < tick; ++t) {
            bool quiet = true;
            for (int c = 0; c < C && quiet; ++c)
                quiet = row[(t - c) % kRing] == 0;
            if (quiet) {
                conv_t = t;
                break;
            }
        }
        const int64_t lp = tick - j->start;
        const bool limit = !j->cur64 && lp >= kRoundPhaseLimit;
        const bool watchdog = j->phases + lp >= cfg.max_phases;
        if (conv_t >= 0 || limit || watchdog) {
            const int64_t ph = conv_t >= 0 ? conv_t + 1 - j->start : lp;
            if (j->round < 4) {
                j->round_ph[j->round] = ph;
                j->round_upd[j->round] = (int64_t)(j->upd - j->upd_round0);
                j->round_state[j->round] = (j->cur64 ? 1 : 0) | (j->in_lds ? 0 : 2) |
                                           (!j->cur64 && j->reg32 ? 4 : 0);
            }
            ++j->round;
            j->phases += ph;
            j->out_of_phases = conv_t < 0 && watchdog;
            conv.push_back(j);
        } else {
            keep.push_back(j);
        }
    }
    running.swap(keep);
    if (!conv.empty()) {
        // the finished requests are not touched again: dicod_poll may free them
        std::vector<Job*> resumed;
        const int rc = check_jobs(conv, resumed);
        running.insert(running.end(), resumed.begin(), resumed.end());
        if (rc != DICOD_OK)
            return rc;
    }
    return DICOD_OK;
}

void server_destroy(Server* s) { delete s; }

int64_t server_open_requests(Server* s)
{
    std::lock_guard<std::mutex> g(s->mu);
    return (int64_t)s->jobs.size();
}

int server_submit(dicod_ctx* ctx, const float* X, int64_t T, double lambda, double eps,
                  int n_seg, uint64_t* req_id)
{
    int K, P, W;
    if (!ctx_dims(ctx, &K, &P, &W))
        return ctx_fail(ctx, DICOD_EINVAL, "dicod_submit: no resident dictionary");
    if (!X || !req_id)
        return ctx_fail(ctx, DICOD_EINVAL, "dicod_submit: NULL argument");
    const dicod_config& cfg = ctx_config(ctx);
    if (T < W)
        return ctx_fail(ctx, DICOD_EINVAL, "dicod_submit: T < W");
    if (T > (int64_t)INT32_MAX / 2)
        return ctx_fail(ctx, DICOD_ENOTSUP, "dicod_submit: T too long");
    if (!std::isfinite(lambda) || lambda == 0.0)
        return ctx_fail(ctx, DICOD_EINVAL, "dicod_submit: lambda must be finite and non-zero");
    if (!(eps > 0.0) || !std::isfinite(eps))
        return ctx_fail(ctx, DICOD_EINVAL, "dicod_submit: eps must be finite and > 0");
    // the server's colours and cap (fixed when it starts)
    Server*& srv = ctx_server(ctx);
    int C = 0, cap_cfg = 0;
    if (srv) {
        C = srv->C;
        cap_cfg = srv->cfg.update_cap;
    } else {
        ctx_serve_schedule(ctx, &C, &cap_cfg);
    }
    const int64_t L = T - W + 1;
    int M = n_seg, tuned = 0;
    if (M < 0)
        return ctx_fail(ctx, DICOD_EINVAL, "dicod_submit: n_seg < 0");
    if (M == 0)
        M = ctx_serve_segments(ctx, L, C, &tuned);
    if (M > L)
        return ctx_fail(ctx, DICOD_EINVAL, "dicod_submit: n_seg > L");
    if (M > 1 && L / M < min_segment_len(W, C))
        return ctx_fail(ctx, DICOD_EINVAL, "dicod_submit: segments shorter than the minimum "
                                           "length for the colour count");
    const int64_t lm = ceil_div(L, M);
    int64_t lx = lm + 2 * (int64_t)(W - 1);
    if (lx > L)
        lx = L;
    const bool fp64 = cfg.precision == DICOD_PREC_FP64;
    // state kernels for float and double rounds (the LDS kernel when allowed
    // and it fits, else the HBM-state kernel)
    auto fits = [&](bool f64, bool* lds) {
        *lds = cfg.state_in_lds && lm <= 4 * kPhaseThreads &&
               lgcd_lds_bytes(K, (int)lm, (int)lx, f64) <= kLdsBytes;
        return *lds || lgcd_gm_lds_bytes(K, (int)lx, f64) <= kLdsBytes;
    };
    bool lds32 = false, lds64 = false;
    if ((!fp64 && !fits(false, &lds32)) || !fits(true, &lds64))
        return ctx_fail(ctx, DICOD_ENOTSUP, "dicod_submit: segments too long for the phase "
                                            "kernels; use more segments");
    if (!srv) {
        Server* ns = new Server();
        const int rc = ns->start(ctx);
        if (rc != DICOD_OK) {
            const std::string m = "dicod_submit: server start: " + ns->fatal_msg;
            delete ns;
            return ctx_fail(ctx, rc, m.c_str());
        }
        srv = ns;
    }
    Job* j = new Job();
    j->T = T;
    j->L = L;
    j->M = M;
    j->lm = (int)lm;
    j->lext = (int)lx;
    j->lam_in = lambda;
    j->eps = eps;
    j->lds32 = lds32;
    j->lds64 = lds64;
    j->tuned = tuned;
    j->reg32 = cfg.reg_state != 0 &&
               lgcd_wave_supported(K, (int)lm, effective_update_cap(cap_cfg, W), false);
    j->lane = M <= kShortSegs ? 0 : 1;
    j->zn = round_up((int64_t)K * L, 64);
    j->xn = round_up((int64_t)P * T, 64);
    if (j->zn > srv->coef.capacity() || j->xn > srv->samp.capacity() || M > srv->seg_cap) {
        delete j;
        std::lock_guard<std::mutex> g(srv->mu);
        return ctx_fail(ctx, DICOD_ENOMEM, "dicod_submit: request larger than the HBM budget");
    }
    const size_t xb = (size_t)P * T * sizeof(float);
    j->hx = (float*)srv->pool.get(xb, &j->hx_cls);
    if (!j->hx) {
        delete j;
        std::lock_guard<std::mutex> g(srv->mu);
        return ctx_fail(ctx, DICOD_ENOMEM, "dicod_submit: pinned host memory exhausted");
    }
    std::memcpy(j->hx, X, xb);
    j->t_submit = now_ms();
    {
        std::lock_guard<std::mutex> g(srv->mu);
        if (srv->fatal != DICOD_OK) {
            srv->pool.put(j->hx, j->hx_cls);
            delete j;
            return ctx_fail(ctx, srv->fatal, ("dicod_submit: " + srv->fatal_msg).c_str());
        }
        j->id = srv->next_id++;
        srv->jobs[j->id] = j;
        srv->queue.push_back(j);
        ++srv->lanes[j->lane].queued;
        ++srv->epoch;
        *req_id = j->id;
    }
    srv->cv.notify_all();
    return DICOD_OK;
}

int server_poll(dicod_ctx* ctx, uint64_t req_id, double* Z_out, dicod_stats* st)
{
    Server* srv = ctx_server(ctx);
    if (!srv)
        return ctx_fail(ctx, DICOD_ENOREQ, "dicod_poll: unknown request");
    Job* j = nullptr;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        auto it = srv->jobs.find(req_id);
        if (it == srv->jobs.end())
            return ctx_fail(ctx, DICOD_ENOREQ, "dicod_poll: unknown request");
        j = it->second;
        if (j->state != kDone)
            return DICOD_PENDING;
        if (!Z_out && j->rc == DICOD_OK)
            return ctx_fail(ctx, DICOD_EINVAL, "dicod_poll: Z_out is NULL");
        j->state = kCopying;
    }
    int rc = j->rc;
    std::string msg = j->err;
    if (Z_out && j->slot >= 0 && (rc == DICOD_OK || rc == DICOD_ENOTCONV)) {
        std::lock_guard<std::mutex> g(srv->copy_mu);
        hipError_t e = hipSetDevice(srv->cfg.device);
        if (e == hipSuccess)
            e = hipMemcpyAsync(Z_out, srv->dZ.as<double>() + j->z_off,
                               (size_t)srv->K * j->L * sizeof(double), hipMemcpyDeviceToHost,
                               srv->cs);
        if (e == hipSuccess)
            e = hipStreamSynchronize(srv->cs);
        if (e != hipSuccess) {
            rc = DICOD_EDEVICE;
            msg = std::string("dicod_poll: copy of Z: ") + hipGetErrorString(e);
        }
    }
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->n_updates = (int64_t)j->upd;
        st->n_phases = j->phases;
        st->n_phase_launches = j->phases;
        st->nnz = (int64_t)j->res.nnz;
        st->n_seg = j->M;
        st->seg_len = (int)(j->L / j->M);
        st->colors = srv->C;
        st->update_cap = srv->cfg.update_cap == 0 ? 0
                                                  : effective_update_cap(srv->cfg.update_cap, srv->W);
        st->tuned = j->tuned;
        {
            // duality gap of the returned Z (as in the one-shot solve)
            const double lam = j->lam;
            const double sc = std::max(lam, j->res.gmax);
            const double primal = 0.5 * j->res.sum_r2 + lam * j->res.l1;
            const double dual = -lam * lam * j->res.sum_r2 / (2.0 * sc * sc) +
                                lam * (j->res.x2 - j->res.bx) / sc;
            st->duality_gap = std::max(primal - dual, 0.0);
            st->n_screened = -1;
        }
        st->converged = j->res.max_dz < j->eps ? 1 : 0;
        st->n_refresh = j->n_refresh;
        st->lambda = j->lam;
        st->lambda_max = j->lmax;
        st->eps = j->eps;
        st->objective = 0.5 * j->res.sum_r2 + j->lam * j->res.l1;
        st->max_dz = j->res.max_dz;
        st->kkt_on = j->res.kkt_on;
        st->kkt_off = j->res.kkt_off;
        st->max_abs_z = j->res.max_abs_z;
        st->t_total_ms = j->t_done - j->t_submit;
        for (int r = 0; r < 4; ++r) {
            st->round_updates[r] = j->round_upd[r];
            st->round_phases[r] = j->round_ph[r];
            st->round_state[r] = j->round_state[r];
            st->round_max_dz[r] = j->round_mdz[r];
        }
        st->state_in_hbm = j->any_hbm ? 1 : 0;
        st->polished_fp64 = j->polished ? 1 : 0;
        st->t_queue_ms = j->t_admit > 0.0 ? j->t_admit - j->t_submit : 0.0;
        st->t_latency_ms = j->t_done - j->t_submit;
    }
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->release(j);
        ++srv->epoch;
        srv->jobs.erase(req_id);
        srv->pool.put(j->hx, j->hx_cls);
        delete j;
        if (rc != DICOD_OK)
            ctx_fail(ctx, rc, msg.c_str());
    }
    srv->cv.notify_all();
    return rc;
}

}  // namespace dicod
