// Internal declarations shared by the HIP translation units of libnbody.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/nbody.h"

// Bits of the device status word latched by kernels.
enum : int {
    NBK_ERANGE = 1,   // a new step fell below dt_min
    NBK_ENAN = 2,     // non-finite acceleration, jerk or step
    NBK_EINDEX = 4,   // active index out of range
};

// Small fixed-size device area of a context (allocated once at creation).
struct nb_small {
    int status;
    int32_t m;
    double t_next;
    double energy[2];
    double blockval[1024];   // per-block minima of t + dt (selection pass 1)
    int32_t blockcnt[1024];  // per-block active counts (selection pass 2)
};

struct nb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    nb_small *small = nullptr;        // device
    nb_small *small_host = nullptr;   // pinned host mirror (only the leading words are used)
    void *scratch = nullptr;          // device, grows on demand
    size_t scratch_bytes = 0;
    std::string err;
};

namespace nbk {

constexpr int WG = 256;          // threads per workgroup (4 waves of 64)
constexpr int SEL_BLOCKS = 1024; // upper bound on selection workgroups

struct ForceArgs {
    const double *xp, *yp, *zp;           // predicted positions (FP64)
    const double *vx64, *vy64, *vz64;     // predicted velocities (FP64 path)
    const double *m64;                    // masses (FP64 path)
    const float *vx32, *vy32, *vz32;      // FP32 copies (mixed path)
    const float *m32;
    const int32_t *i_idx;                 // active list, or null for i = k
    int32_t m;                            // active block size
    int64_t n;                            // bodies in the system (index bound)
    int64_t j0, j1;                       // j-range
    int64_t chunk;                        // j per workgroup chunk (multiple of the tile)
    double eps2;
    double *out_acc, *out_jerk;           // rows c*m + k, plus b*stride_b
    int64_t stride_b;
    int *status;
};

// Launch one force kernel instance; returns hipSuccess or the launch error.
hipError_t launch_force(int precision, int il, int s, dim3 grid, const ForceArgs &a,
                        hipStream_t st);
// out[c*m+k] = sum_b part[b*6m + c*m + k] in ascending b, for c < 6.
hipError_t launch_reduce_partials(const double *part, int32_t m, int nb, double *acc,
                                  double *jerk, hipStream_t st);
// Energy: per-body m_i * sum_{j != i} m_j / sqrt(r^2 + eps^2) into rows[n], then
// compensated totals (kinetic, potential) into out[2].
hipError_t launch_energy(const nb_system &s, double eps2, double *rows, double *out,
                         hipStream_t st);

// Step kernels.
hipError_t launch_select(const nb_system &s, nb_small *small, int32_t *i_idx, hipStream_t st);
hipError_t launch_predict(const nb_system &s, double t_next, hipStream_t st);
hipError_t launch_correct(const nb_system &s, const int32_t *i_idx, int32_t m,
                          const double *acc, const double *jerk, double t_next, double eta,
                          double dt_max, double dt_min, int *status, hipStream_t st);
hipError_t launch_init_steps(const nb_system &s, const double *acc, const double *jerk,
                             double eta_s, double dt_max, double dt_min, int *status,
                             hipStream_t st);

}  // namespace nbk
