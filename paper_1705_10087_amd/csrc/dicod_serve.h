// Serving loop of the LGCD library (continuous batching of encode requests).
#pragma once

#include <cstdint>

#include "dicod.h"

namespace dicod {

struct Server;

void server_destroy(Server* s);
// Requests submitted and not yet returned by dicod_poll.
int64_t server_open_requests(Server* s);
int server_submit(dicod_ctx* ctx, const float* X, int64_t T, double lambda, double eps,
                  int n_seg, uint64_t* req_id);
int server_poll(dicod_ctx* ctx, uint64_t req_id, double* Z_out, dicod_stats* st);

// Device pointers of the resident dictionary (read-only while serving).
struct DictView {
    const double* D64;                 // [K][P][W]
    const double* S64;                 // [l][k][d] double
    const void* S32;                   // [l][k][d] float
    const void* St32;                  // phase-kernel layout, float
    const void* St64;                  // phase-kernel layout, double
    const double* Sc64;                // [l][k][2W] double, the check's copy
    const void *n2_32, *inv32, *n2_64, *inv64;
    const unsigned short* Dsp;         // bf16 hi/lo split of D (split-bf16 correlation)
    double dnorm_max;                  // max_k |D_k|
};

// accessors implemented in dicod_api.cpp
Server*& ctx_server(dicod_ctx* ctx);
const dicod_config& ctx_config(const dicod_ctx* ctx);
int ctx_dims(const dicod_ctx* ctx, int* K, int* P, int* W);
DictView ctx_dict(const dicod_ctx* ctx);
int ctx_fail(dicod_ctx* ctx, int code, const char* msg);

// Segment-length rules shared with the one-shot solver.
int64_t min_segment_len(int W, int C);
int auto_segment_count(int64_t L, int W, int C);
// Schedule of a server from the tuning table (autotune on) or the config.
void ctx_serve_schedule(const dicod_ctx* ctx, int* colors, int* update_cap);
// Segment count of a request of L coefficients under C colours.
int ctx_serve_segments(const dicod_ctx* ctx, int64_t L, int C, int* tuned);

}  // namespace dicod
