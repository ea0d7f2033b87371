// Internal declarations shared by the host runtime (dicod_api.cpp) and the
// gfx950 kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dicod.h"

namespace dicod {

constexpr int kCheckKB = 8;      // most atoms of one block of the double check
constexpr int kCheckSpan = 1024; // positions of one tile of the double check
constexpr int kCheckParts = 10;  // partials per check tile
constexpr int kMaxP = 16;        // channels accepted (the correlation kernels stage P rows)
constexpr int kPhaseThreads = 512;
constexpr int kPhaseThreadsMax = 1024;
constexpr int kMaxColors = 4;  // phase classes of the segment schedule
constexpr int kTile = 256;       // positions per workgroup in the tiled kernels
constexpr int kAbsChunk = 4096;  // [K][L] elements per workgroup in the max kernels
constexpr size_t kLdsBytes = 163840;  // LDS per workgroup on gfx950
constexpr int kRunUpdateBound = 1 << 16;  // updates per segment run when uncapped
constexpr int64_t kRoundPhaseLimit = 4096; // float descent phases between checks

// One signal of a (possibly batched) solve.
struct SigDesc {
    int64_t x_off;    // element offset of X_i ([P][T] row-major)
    int64_t z_off;    // element offset of the [K][L] arrays (g, Z, beta0)
    int64_t T;        // samples
    int64_t L;        // T - W + 1
    int32_t seg_base; // global index of its first segment
    int32_t M;        // number of segments
    double lam;       // lambda used
    double eps_stop;  // a segment run stops when its best |Delta Z| is below this
    int64_t nz_off;   // first word of its non-zero masks of Z ([K][ceil(L / 64)])
};

// One time segment C_m of one signal.
struct SegDesc {
    int64_t z_off;  // element offset of the signal's [K][L] arrays
    int32_t L;      // signal length in coefficients
    int32_t b, e;   // segment covers t in [b, e)
    int32_t sig;    // signal index
    int32_t left;   // neighbour segment indices, -1 at the signal ends
    int32_t right;
};

// Updates per segment run: update_cap > 0 as given, 0 = no cap (a bound that
// still ends every run), -1 = max(4, round(2 sqrt(W))) (measured: 28 at
// W = 200, 16 at W = 64).
int effective_update_cap(int update_cap, int W);

// Per-signal results of the double-precision check, reduced from partials.
struct CheckResult {
    double max_dz;
    double kkt_on;
    double kkt_off;
    double l1;
    double sum_r2;
    double max_abs_z;
    double nnz;
    double bx;         // <beta0, Z> = <X, sum_k Z_k * D_k>
    double gmax;       // max |g| = max |D^T R| over the coordinates
    double x2;         // |X|^2
    double pad;
};

// Device-side counters of one solve.
struct Counters {
    unsigned long long seg_runs;   // segment runs that made at least one update
    unsigned long long trace_n;    // trace records requested
    unsigned long long box_overflow;  // boundary records that found a full mailbox or ring
    unsigned long long upd_seq;    // free-running schedule: updates numbered in selection order
};

// A boundary update of the coloured schedule with mailboxes (register-state
// kernel): the update (k0, t0, delta) of a segment whose window reaches a
// neighbour, applied by that neighbour when it next runs (the message of
// Algorithm 2, delivered before the receiver's next run).
struct BoundaryRec {
    int32_t k0;
    int32_t t0;     // position in the signal
    float delta;
    int32_t seq;    // free-running schedule with a trace: the update's number; else 0
};

// Static device scratch of dicod_solve_device_noalloc (noalloc.hip): its size,
// and its device address on `device` (which must be the current device),
// looked up once per device with hipGetSymbolAddress.
size_t scratch_bytes();
hipError_t scratch_address(int device, void** out);

// ---- launchers (kernels.hip) ------------------------------------------------
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, size_t n,
                           hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, size_t n, hipStream_t s);

// out[b][k][t] = sum_{p,tau} D[k][p][tau] Y_b[p][t + tau] in double on MFMA
// (f64 16x16x4).  Signals/tiles are described by sig[] and tile_pref[].
// z0 / z32_0 (may be NULL): zeroed at every output coordinate (the descent's
// Z and its float copy); amax_bits (may be NULL): per signal, atomic maximum
// of the bits of max |out| (the caller zeroes it first).
hipError_t launch_corr_f64_x32(const double* D, int K, int P, int W, const float* Y,
                               const SigDesc* sig, const int64_t* tile_pref,
                               int n_sig, int64_t n_tiles, double* out64,
                               float* g32, double* g64, hipStream_t s, double* z0 = nullptr,
                               float* z32_0 = nullptr, unsigned long long* amax_bits = nullptr);
hipError_t launch_corr_f64_x64(const double* D, int K, int P, int W,
                               const double* Y, const SigDesc* sig,
                               const int64_t* tile_pref, int n_sig,
                               int64_t n_tiles, double* out64, hipStream_t s);
// Same contraction in float with split bf16 on MFMA (16x16x32 bf16, fp32
// accumulation of hi*hi + hi*lo + lo*hi); Dsp from launch_split_d.
hipError_t launch_corr_bf16x3(const unsigned short* Dsp, int K, int P, int W, const float* Y,
                              const SigDesc* sig, const int64_t* tile_pref, int n_sig,
                              int64_t n_tiles, float* g32, hipStream_t s);
// Dsp = {hi, lo}[p][Kp][Wp] bf16 split of D float [K][P][W] (Kp, Wp: K and W
// rounded up to multiples of 32, zero padded); corr_bf16_dsp_elems elements.
size_t corr_bf16_dsp_elems(int K, int P, int W);
hipError_t launch_split_d(const float* D, int K, int P, int W, unsigned short* Dsp,
                          hipStream_t s);

// Dictionary finish: S32 = (float)S64, n2 = S64[k][k][W-1], inverses.
hipError_t launch_dict_finish(const double* S64, int K, int W, float* S32,
                              double* n2_64, double* inv_n2_64, float* n2_32,
                              float* inv_n2_32, hipStream_t s);

// Per-signal max |beta| as the bit pattern of a non-negative double.
hipError_t launch_absmax(const double* beta, int K, const SigDesc* sig,
                         const int64_t* tile_pref, int n_sig, int64_t n_tiles,
                         unsigned long long* out_bits, hipStream_t s);

// A boundary message of Algorithm 2: the neighbour's update (k0, t0, delta).
struct DicodMsg {
    int32_t k0;
    int32_t t0;     // position in the signal
    double delta;   // applied change of Z_{k0}[t0]
};

// One phase of locally greedy CD over the segments in list[].
struct PhaseArgs {
    const SegDesc* segs;
    const int32_t* list;
    int n_list;
    void* g;              // float or double state [K][L] per signal
    double* Z;            // double [K][L] per signal
    const void* S;        // [K][K][2W-1] in the state's type
    const void* n2;       // [K]
    const void* inv_n2;   // [K]
    const SigDesc* sigs;
    int K, W, cap;
    int phase;
    int phase_stride;     // per-signal rows of phase_upd (0: one row for all)
    uint32_t* dirty;
    unsigned long long* phase_upd;  // [sig * phase_stride + phase] updates
    unsigned long long* sig_upd;   // per-signal applied updates
    int* sig_last_upd;
    Counters* counters;
    dicod_trace_rec* trace;
    long long trace_cap;
    int lm_max, lext_max;
    // Algorithm 2 in lockstep (schedule DICOD): every segment keeps only its
    // own positions, applies the messages its neighbours sent in the previous
    // phase and sends its own; dirty flags and message boxes are
    // double-buffered by phase parity.
    int dicod;              // 1 = this schedule (LDS-state kernel only)
    int n_seg;              // segments in the table: stride of dirty[] and boxes
    int msg_cap;            // messages per box (>= cap)
    DicodMsg* msg;          // [2 parity][n_seg][2: 0 leftwards, 1 rightwards][msg_cap]
    uint32_t* msg_n;        // [2 parity][n_seg][2]
    // Register-state kernel: boundary mailboxes box[s][side][box_cap] with
    // counts box_n[s][side] (side 0: records from the left neighbour, 1: from
    // the right one), and a float copy of Z (z32, same layout as Z) from which
    // the run loads its state.
    BoundaryRec* box;
    uint32_t* box_n;
    int box_cap;
    float* z32;
    // Set to 1 for every segment whose Z a run changed (the double check
    // recomputes only the tiles within reach of such segments); may be null.
    uint32_t* changed;
};
hipError_t launch_lgcd_phase(const PhaseArgs& a, bool fp64, size_t* lds_bytes,
                             hipStream_t s);
size_t lgcd_lds_bytes(int K, int lm_max, int lext_max, bool fp64);
// The same phase with g and Z kept in HBM (segments too long for LDS, or
// double state at large K * W); S in the [l][k][d] layout.
hipError_t launch_lgcd_phase_gm(const PhaseArgs& a, bool fp64, size_t* lds_bytes,
                                hipStream_t s);
size_t lgcd_gm_lds_bytes(int K, int lext_max, bool fp64);
// Float phase with each position's state in the registers of one thread
// (lgcd_wave.hip): segments of at most 256 positions, K <= 32, at most 64
// updates per run, coloured schedule; S in the phase-kernel layout
// (launch_s_transpose, float).
bool lgcd_wave_supported(int K, int lm_max, int cap, bool fp64);
// Mailbox capacity (records per segment and side) the kernel needs: a.box_cap.
int lgcd_wave_box_cap();
hipError_t launch_lgcd_wave(const PhaseArgs& a, hipStream_t s);

// Free-running schedule (Algorithm 2 without phase barriers, lgcd_async.hip):
// persistent teams, each looping over the segments sid = team, team +
// n_teams, ... for up to `sweeps` passes; a segment runs when it has work
// (dirty) or records waiting, and boundary records travel through
// single-producer rings ring[s][side][ring_cap] with monotone counters
// ring_w (records written, advanced by the neighbour with release order) and
// ring_r (records applied, advanced by the owner).  A team stops early after
// a pass in which none of its segments ran.  No team ever waits for another.
constexpr int kAsyncSweeps = 4;  // passes over the segments per free-running launch
struct AsyncArgs {
    BoundaryRec* ring;
    uint32_t* ring_w;     // [n_seg][2]
    uint32_t* ring_r;     // [n_seg][2]
    int ring_cap;
    int sweeps;
    int n_teams;
};
// Ring capacity for a given update cap and sweeps per launch: records of one
// launch plus those left from the previous one.
int lgcd_async_ring_cap(int cap, int sweeps);
// Teams of the free-running launch for these segments (at most the resident
// capacity of the device).
int lgcd_async_teams(int K, int lm_max, int n_seg, int n_cu);
hipError_t launch_lgcd_async(const PhaseArgs& a, const AsyncArgs& x, hipStream_t s);
// Atoms per position in the phase kernel's layout (K padded), -1 if K is
// beyond the instantiated sizes.
int lgcd_k_padded(int K, bool fp64);
// St[l][d][k] = S_{k,l}[d - W + 1] (k < K; 0 for padded atoms), float or double.
hipError_t launch_s_transpose(const double* S64, int K, int W, bool fp64, void* St,
                              hipStream_t s);

// Non-zero masks of Z for the check kernels: bit i of word
// masks[sig.nz_off + k * ceil(L / 64) + b] tells Z_k[64 b + i] != 0.
// mask_pref: prefix of the signals' word counts (n_sig + 1 entries).
hipError_t launch_nz_mask(const double* Z, const SigDesc* sig, const int64_t* mask_pref,
                          int n_sig, int K, int64_t n_words, unsigned long long* masks,
                          hipStream_t s);
// Double-precision stop test and refresh: g = beta0 - S * Z from the
// non-zeros of Z (masks from launch_nz_mask) or the maintained double state
// g_in, Delta Z of every coordinate in double, the optimality residuals, the
// objective partials |X|^2 and <beta0 + g, Z> (their difference is
// |X - Z * D|^2), dirty flags for segments holding a coordinate with
// |Delta Z| >= flag_eps, and an optional refresh of the state g (float or
// double) and of the float copy z32 of Z (when not NULL).  Tiles of kCheckSpan positions (tile_pref: prefix of
// ceil(L / kCheckSpan)); part: [check_kblocks(K, W)][n_tiles][kCheckParts].
// Sc: the padded copy of S described at check_s_elems.
hipError_t launch_grad_check(const float* X, const double* beta0, const double* Z,
                             const unsigned long long* masks, const double* Sc,
                             const double* n2, int K, int P, int W, const SigDesc* sig,
                             const int64_t* tile_pref, int n_sig, int64_t n_tiles,
                             double flag_eps, const uint32_t* sig_done, uint32_t* dirty,
                             void* g_state, bool state_fp64, const double* g_in,
                             double* part, float* z32, const uint32_t* changed, hipStream_t s);
// (changed, when not NULL: per-segment flags of Z changed since the last
// check; a tile whose reach holds no changed segment keeps its partials and
// refreshed state from that check, which must have run on the same tiles with
// the same state output, and only re-marks its segments dirty.)
// Atom blocks of the check (grid y); 0 when W is too large for it.
int check_kblocks(int K, int W);
int check_atoms_per_block(int K, int W);
// Sc: S in the [l][k][2W] layout (row d = 0..2W-2, one pad element per row)
// followed by 128 doubles of padding; check_s_elems(K, W) elements.
size_t check_s_elems(int K, int W);
hipError_t launch_check_reduce(const double* part, const int64_t* tile_pref, int64_t n_tiles,
                               int n_kblk, int n_sig, CheckResult* out, hipStream_t s);

// MIXED precision: gather candidates with |beta| >= thr and recompute them in
// double; per-signal max of the exact values.
hipError_t launch_refine_absmax(const float* beta32, const double* D, const float* X,
                                int K, int P, int W, const SigDesc* sig,
                                const int64_t* tile_pref, int n_sig, int64_t n_tiles,
                                const double* thr, unsigned long long* out_bits,
                                hipStream_t s);
// Per signal, max over t < L of sum_p sum_{tau < W} X[p][t + tau]^2 (bits of a
// non-negative double, atomic max; out_bits zeroed by the caller).  Tiles of
// kTile positions (tile_pref: prefix of ceil(L / kTile)).  For W up to about
// 20,000 (LDS).
size_t win_energy_lds_bytes(int W);
hipError_t launch_win_energy_max(const float* X, int P, int W, const SigDesc* sig,
                                 const int64_t* tile_pref, int n_sig, int64_t n_tiles,
                                 unsigned long long* out_bits, hipStream_t s);
// Coordinates proved zero by the Gap Safe rule (kernels.hip): g float or
// double [K][L] per signal, rule[2 i] = 1 / max(lambda, max|g|) and
// rule[2 i + 1] = sqrt(2 gap) / lambda; count per signal (accumulated).
hipError_t launch_screen_count(const void* g, bool fp64, const double* n2, int K,
                               const SigDesc* sig, const int64_t* tile_pref, int n_sig,
                               int64_t n_tiles, const double* rule, unsigned long long* count,
                               hipStream_t s);
// Candidate threshold of the refinement per signal (lambda_bound.hip):
// thr[i] = max(0, v_i - 2 coef sqrt(e_i)) from the bits of the largest split
// |beta| v_i and the largest window energy e_i; coef = refine_coef(P, W,
// max_k |D_k|) = 1.05 (3.1 2^-16 + (P W + 1) 2^-24) max_k |D_k|.
double refine_coef(int P, int W, double dnorm_max);
hipError_t launch_refine_threshold(const unsigned long long* vbits,
                                   const unsigned long long* ebits, int n, double coef,
                                   double* thr, hipStream_t s);
hipError_t launch_absmax_f32(const float* beta, int K, const SigDesc* sig,
                             const int64_t* tile_pref, int n_sig, int64_t n_tiles,
                             unsigned long long* out_bits, hipStream_t s);

// Serving: tab[slots[i]].lam = lam_in[i] (> 0) or -lam_in[i] * lambda_max[i].
hipError_t launch_apply_lambda(SigDesc* tab, const int* slots, const double* lam_in,
                               const unsigned long long* lmax_bits, int n, hipStream_t s);
// tab[0..n).eps_stop = eps (the stop threshold of the descent state).
hipError_t launch_set_eps_stop(SigDesc* tab, int n, double eps, hipStream_t s);
// dirty[i] = 0 for every segment i < n_seg whose signal has done[sig] != 0.
hipError_t launch_clear_done_dirty(const SegDesc* segs, int n_seg, const uint32_t* done,
                                   uint32_t* dirty, hipStream_t s);
// Serving: ring[r][(start + c) % H] = 0 for r < rows, c < n.
hipError_t launch_clear_ring(unsigned long long* ring, int rows, int H, int start, int n,
                             hipStream_t s);

}  // namespace dicod
