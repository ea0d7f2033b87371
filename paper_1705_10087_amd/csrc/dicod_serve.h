// Serving loop of the LGCD library (continuous batching of encode requests).
#pragma once

#include <cstdint>

#include "dicod.h"

namespace dicod {

struct Server;

void server_destroy(Server* s);
int server_submit(dicod_ctx* ctx, const float* X, int64_t T, double lambda, double eps,
                  int n_seg, uint64_t* req_id);
int server_poll(dicod_ctx* ctx, uint64_t req_id, double* Z_out, dicod_stats* st);

// accessors implemented in dicod_api.cpp
Server*& ctx_server(dicod_ctx* ctx);
const dicod_config& ctx_config(const dicod_ctx* ctx);
int ctx_dims(const dicod_ctx* ctx, int* K, int* P, int* W);
int ctx_fail(dicod_ctx* ctx, int code, const char* msg);

}  // namespace dicod
