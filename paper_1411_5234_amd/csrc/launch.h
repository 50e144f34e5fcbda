// Host-side launchers of the kernels of libnbody.so (each defined beside its
// kernel); called by the C ABI in api.hip.
#pragma once

#include "nb_internal.h"

namespace nbk {

// Force kernels for one plan shape (IL i-bodies per lane, S lanes per i-body).
hipError_t launch_force(int precision, int il, int s, const Table &t, hipStream_t st);
// 6th order: acceleration, jerk and snap.
hipError_t launch_force6(int precision, int il, int s, const Table &t, hipStream_t st);
// out[c*m + k] = sum_b part[b*K*m + c*m + k] (K = force_outputs) in the fixed
// order of reduce_partials_kernel, written to acc, jerk (and snap).
hipError_t launch_reduce(const Table &t, hipStream_t st);
// Energy of one system: rows[i] = m_i sum_{j != i} m_j / sqrt(r^2 + eps^2), then
// compensated totals (kinetic, potential) into out[2].
hipError_t launch_energy(const nb_system &s, double eps2, double *rows, double *out,
                         hipStream_t st);

// Tidal tensors of the listed bodies, one workgroup per body, rows (3a+b)*m + k.
hipError_t launch_tidal(const Table &t, hipStream_t st);
hipError_t launch_nearest(const Table &t, hipStream_t st);
// Selection: two passes over per-item workgroup slices, then per-item results.
hipError_t launch_select(const Table &t, double *blockval, int32_t *blockcnt, SelResult *res,
                         hipStream_t st);
// Copy `bytes` (a multiple of 16) from mapped pinned host memory `src` (its
// device address) to device memory `dst`, in stream order.
hipError_t launch_upload(const char *src, char *dst, size_t bytes, hipStream_t st);
// Copy each item's status word into res[k].status, then clear the words; host
// (mapped pinned memory, or null) also receives every item's whole result, and
// then, when `flag` (mapped pinned memory) is set, the value `seq` in *flag.
hipError_t launch_collect_status(const Item *items, int n, SelResult *res, SelResult *host,
                                 unsigned *flag, unsigned seq, hipStream_t st);
// sel: null, or the device selection results of the same items (see predict_kernel).
hipError_t launch_predict(const Table &t, const SelResult *sel, hipStream_t st);
hipError_t launch_correct(const Table &t, double eta, double dt_max, double dt_min,
                          hipStream_t st);
hipError_t launch_init_steps(const Table &t, double eta_s, double dt_max, double dt_min,
                             hipStream_t st);
hipError_t launch_predict6(const Table &t, const SelResult *sel, hipStream_t st);
hipError_t launch_correct6(const Table &t, double eta, double dt_max, double dt_min,
                           hipStream_t st);
hipError_t launch_init_steps6(const Table &t, double eta_s, double dt_max, double dt_min,
                              hipStream_t st);

}  // namespace nbk
