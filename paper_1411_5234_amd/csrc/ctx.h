// The host-side context of libnbody.so (nb_ctx): stream, scratch buffers, the
// item-table upload ring, side streams and the pair-advance worker thread.
// Host code only; the kernels see nb_internal.h.
#pragma once

#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <string>
#include <thread>

#include "nb_internal.h"

struct nb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    nb_small *small = nullptr;        // device
    nb_small *small_host = nullptr;   // pinned host mirror
    void *scratch = nullptr;          // device: force partials, energy rows (grows)
    void *noalloc_area = nullptr;     // device address of the static area on this device
    size_t scratch_bytes = 0;
    void *selbuf = nullptr;           // device: selection per-workgroup temporaries (grows)
    size_t selbuf_bytes = 0;
    void *res = nullptr;              // device: per-item selection results (grows)
    void *res_host = nullptr;         // pinned, mapped: the results as the host reads them
    void *res_host_dev = nullptr;     // device address of res_host
    size_t res_bytes = 0;
    char *stage_host = nullptr;       // pinned, mapped, coherent ring for item tables
    const char *stage_host_dev = nullptr;   // device address of stage_host
    char *stage_dev = nullptr;        // device ring mirrored by stage_host
    size_t stage_bytes = 0, stage_off = 0;
    std::string err;
    // Side streams (default priority, created on first use) on which force
    // launches of different plan shapes in one call run beside the one on
    // `stream`, forked from and joined back to it with events.
    static constexpr int NSIDE = 3;
    hipStream_t side[NSIDE] = {};
    hipEvent_t fork = nullptr, join[NSIDE] = {};
    bool side_ready = false;
    // Sequence number the status kernel writes into the flag word after the results.
    unsigned sel_seq = 0;
    // Host thread for pair advances (started on first use): a FIFO of jobs run in
    // call order; result is the first failure since the last wait.
    struct Worker {
        std::thread th;
        std::mutex mu;
        std::condition_variable cv;
        std::deque<std::function<int()>> queue;
        bool running = false, quit = false;
        int result = 0;
    } worker;
};

// Pair advance (csrc/groups.hip); async = queue on the context's thread.
nb_status nb_groups_run(nb_ctx *ctx, int32_t n, const int32_t *idx, const double *M, double *r,
                        double *v, const double *H, const double *T0, const double *T1,
                        int32_t per_period, int64_t max_sub, int32_t *status, bool async);

