// Library handle: stream, device, pinned read-back buffer and the device
// workspace arena shared by every call made with the handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

struct zolo_handle_s {
    hipStream_t stream = nullptr;
    int device = 0;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    double* host = nullptr;  // pinned scalars for read-back
    int panel_coresident = 0;
    float* est = nullptr;    // learned l/r estimator parameters (zolo_set_estimator)
    // Worker handles of zolo_pd_batched: cooperative panel launches go to the
    // shared panel stream (one panel in flight at a time across workers),
    // ordered against this handle's stream by the two events.
    hipStream_t panel_stream = nullptr;
    hipEvent_t ev_ready = nullptr, ev_done = nullptr;
    // Solves of zolo_pd_batched (sequential or concurrent alike, so that
    // both give the same bits): panels of few rows take one workgroup.
    bool single_panels = false;
    // zolo_pd_batched's workers, created on its first call with several
    // streams and kept (streams, pinned buffers, events, workspaces grown on
    // demand) until zolo_destroy; the shared stream of their cooperative
    // panels.
    std::vector<zolo_handle_s*> workers;
    hipStream_t worker_panel_stream = nullptr;
    // Second stream of the QR look-ahead (structured_geqrf), created by the
    // first zolo_pd call (never by zolo_pd_noalloc), with its two events.
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_side_ready = nullptr, ev_side_done = nullptr;
};
