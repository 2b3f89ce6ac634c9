// Kernel argument blocks and launchers of the SB solver (host <-> device).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sbt {

constexpr int kEnergyRows = 64;  // rows per workgroup in energy_rows

struct ResidentArgs {
    int n, nnz, M, K;
    int ckpt_every;              // > 0: FP64 energy every that many steps
    double a0;
    float dt, dta0;
    const int *row_ptr;          // [n+1]
    const int *col;              // [nnz]
    const float *J;              // [nnz] FP32 couplings
    const float *h;              // [n]   FP32 field
    const double *scal;          // [0] = c0
    const double *a;             // [n]   FP64 QUBO (checkpoint energies)
    const double *b;             // [nnz]
    float *x;                    // [n*M] in: start, out: final
    float *y;                    // [n*M]
    double *etrace;              // [n_ckpt*M]
    const int *perm;             // [n] spin order (register-row variant)
    const float *sched;          // [K] a0 - a_k (schedule table)
};

struct ResidentShape {
    int tpb;                     // threads per workgroup (register-row variant: any
                                 //   multiple of 64 up to 1024)
    int spt;                     // spins per thread: 1, 2, 4, 8 (16 for the LDS-row variant)
    int rc;                      // > 0: register-row variant with this many couplings per
                                 //   row in VGPRs (2, 4, 8); 0: LDS-row variant
    bool jlds;                   // LDS-row variant: J held in LDS
    size_t lds_bytes;
};

constexpr int kRegMaxN = 8192;   // register-row variant: largest n (buffer stride)

struct StreamArgs {
    int n, M, K;
    double a0;
    float dt, dta0;
    const int *row_ptr;
    const int *col;
    const float *J;
    const float *h;
    const double *scal;
    float *y;
    const float *sched;          // [K] a0 - a_k
};

hipError_t launch_prep(int n, const double *a, const int *row_ptr, const int *col, const double *b,
                       float *J, float *h, double *part, double *scal, double c0_fixed,
                       hipStream_t st);
hipError_t launch_init(int n, int M, uint64_t seed, uint32_t event, float *x, float *y,
                       hipStream_t st);
hipError_t launch_schedule(int K, double a0, float *sched, hipStream_t st);
hipError_t launch_resident(int mode, const ResidentArgs &A, const ResidentShape &S, hipStream_t st);
hipError_t launch_resident_reg(int mode, const ResidentArgs &A, const ResidentShape &S,
                               hipStream_t st);
hipError_t launch_row_order(int n, const int *row_ptr, int *perm, hipStream_t st);
hipError_t launch_stream_step(int mode, const StreamArgs &A, int k, const float *xin, float *xout,
                              hipStream_t st);
hipError_t launch_energy(int n, int M, const double *a, const int *row_ptr, const int *col,
                         const double *b, const float *x, double *part, double *out,
                         hipStream_t st);
hipError_t launch_select_best(int n, int M, const double *E, const float *x, double *best_e,
                              int *best_m, int8_t *T, hipStream_t st);
hipError_t launch_trace_reduce(int n_ckpt, int M, const double *et, double *trace, hipStream_t st);

}  // namespace sbt
