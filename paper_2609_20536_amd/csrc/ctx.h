// Library context shared by the run engine and the surrogate: device,
// stream, workspace, per-run step logs, timing events and pinned staging.
#pragma once

#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

namespace gxy {

struct RunLog {
  std::vector<gxy_step_info> steps;
};

}  // namespace gxy

struct gxy_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  std::string last_error;
  std::vector<gxy::RunLog> logs;
  double phase_ms[6] = {0, 0, 0, 0, 0, 0};
  // per-launch events around the dominant contraction (the D^7 product)
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, double>> hot_launches;  // (event pair index, flops)
  double hot_stats[4] = {0, 0, 0, 0};  // launches, ms, flops, bytes
  bool hot_on = false;
  void *pinned = nullptr;  // small host staging buffer
  size_t pinned_bytes = 0;
  // two pinned staging buffers for table uploads, each guarded by an event
  void *stage[3] = {nullptr, nullptr, nullptr};
  size_t stage_bytes[3] = {0, 0, 0};
  hipEvent_t stage_ev[3] = {nullptr, nullptr, nullptr};
  bool stage_used[3] = {false, false, false};
  // pinned arenas for the projection tables of a step, by step parity
  void *arena[2] = {nullptr, nullptr};
  size_t arena_bytes[2] = {0, 0};
  bool arena_pageable[2] = {false, false};  // arena[q] lives in arena_host[q]
  std::vector<char> arena_host[2];
  hipEvent_t arena_ev[2] = {nullptr, nullptr};
  bool arena_pending[2] = {false, false};
  // second stream for the impurity projections, and the events that order
  // it against the main stream (slots: see run_one)
  hipStream_t imp_stream = nullptr;
  hipEvent_t pipe_ev[8] = {nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, nullptr};
  hipEvent_t sel_ev = nullptr;  // selection results copied to the host
  // side stream for the projection table copies, with one event per launch
  hipStream_t copy_stream = nullptr;
  std::vector<hipEvent_t> copy_ev;
  // projection tile per Dcut chosen by gxy_autotune (absent: by tile fill);
  // force_tile (64 / 128) overrides both while the autotuner measures
  std::map<int, int> tile_for_dcut;
  int force_tile = 0;
  bool hot_force = false;  // keep the contraction events on (autotuner)
  // batched runs: worker contexts, each with its own stream and workspace
  int batch_workers = 0;  // 0 = default
  size_t chunk_bytes = 0;  // projection chunk bound (0: GXY_CHUNK_BYTES or 32 GiB)
  bool worker = false;     // batch worker: one stream, no side streams
  std::vector<gxy_ctx *> children;
  // no-allocation runs (gxy_run_noalloc): this device's address of the
  // library's static scratch array (looked up once per device at
  // gxy_create), the flag that routes a run through it with one stream and
  // no HIP allocation, and fixed host staging for results read back
  void *scratch = nullptr;
  bool noalloc = false;
  std::vector<char> noalloc_arena;          // projection tables (host planning)
  alignas(64) unsigned char noalloc_host[1 << 20];
};

// Every C entry point runs its body inside these: library errors become
// status codes and the message is kept for gxy_last_error.
#define GXY_API_BEGIN try {
#define GXY_API_END(ctx)                                         \
  }                                                              \
  catch (const Error &e) {                                       \
    if (ctx) (ctx)->last_error = e.msg;                          \
    if (getenv("GXY_LOG")) fprintf(stderr, "gxy: %s\n", e.msg.c_str()); \
    return e.status;                                             \
  }                                                              \
  catch (const std::bad_alloc &) {                               \
    if (ctx) (ctx)->last_error = "host allocation failed";       \
    return GXY_ENOMEM;                                           \
  }                                                              \
  catch (...) {                                                  \
    if (ctx) (ctx)->last_error = "unexpected host exception";    \
    return GXY_EDEVICE;                                          \
  }
