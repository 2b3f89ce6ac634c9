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
    int spt;                     // spins per thread: register-row 1, 2, 3, 4, 8; LDS-row a
                                 //   power of two up to 16
    int rc;                      // > 0: register-row variant with this many couplings per
                                 //   row in VGPRs (2, 4, 8) for slot 0; 0: LDS-row variant
    int rr;                      // register-row variant: couplings in VGPRs per row of the
                                 //   other slots (rc, or 2)
    bool jlds;                   // LDS-row variant: J held in LDS
    size_t lds_bytes;
};

// Register-row variant: VGPR estimate of a thread holding spt spins, rc
// couplings in registers for slot 0 and rr for each other slot (fit to the
// compiler's counts), the budget at a workgroup size, and which shapes
// exist -- the host picks a shape only among these.  Slot 0 holds the
// longest rows, so when the same capacity for every slot does not fit, the
// other slots get 2 (rows longer than a slot's capacity continue from
// global memory).
constexpr int reg_vgpr_estimate(int spt, int rc, int rr) {
    return 4 * (rc + (spt - 1) * rr) + 12 * spt + 40;
}
constexpr int reg_vgpr_budget(int maxtpb) { return maxtpb >= 1024 ? 128 : (maxtpb >= 512 ? 256 : 512); }
constexpr bool reg_fits(int maxtpb, int spt, int rc, int rr) {
    return !(spt > 4 && rc > 4) && reg_vgpr_estimate(spt, rc, rr) <= reg_vgpr_budget(maxtpb);
}
// the shapes that are built: same capacity everywhere where it fits, else
// (rc, 2) where that fits with kSplitSlack VGPRs to spare (the compiler
// keeps the step loop of such shapes spill-free -- checked on the ISA of
// (1024 threads, 4 spins, 8/2) -- spilling only in the code around it)
constexpr int kSplitSlack = 16;
constexpr bool reg_variant_fits(int maxtpb, int spt, int rc, int rr) {
    if (rr == rc) return reg_fits(maxtpb, spt, rc, rc);
    return spt > 1 && rr == 2 && rc > 2 && !reg_fits(maxtpb, spt, rc, rc) && !(spt > 4 && rc > 4) &&
           reg_vgpr_estimate(spt, rc, 2) <= reg_vgpr_budget(maxtpb) + kSplitSlack;
}

constexpr int kRegMaxN = 8192;   // register-row variant: largest n
constexpr int kRegTailCap = 1792;  // register-row variant: couplings past the rows'
                                   //   register capacity staged in LDS (14 KB)
constexpr int kRegStride = kRegMaxN + 64;  // LDS position buffer: n words, then one pad
                                           //   word per lane of a wave

// ---------------------------------------------------------------- batch

constexpr int kBatchTPB = 1024;                     // threads per workgroup, large shape
constexpr int kBatchTPBSmall = 512;                 // small shape (two workgroups per CU)
constexpr int kBatchSPT = 9;                        // slots per thread (both shapes)
constexpr int kBatchSlots = kBatchTPB * kBatchSPT;  // largest n * agents per item
constexpr int kBatchSlotsSmall = kBatchTPBSmall * kBatchSPT;
constexpr int kBatchTailCap = 8192;                 // default LDS words for couplings past the
                                                    //   slots' register capacity (32 KB)
// coupling formats: 16-bit (batch), FP32, FP8 e4m3 with a per-row scale,
// FP8 e4m3 with a per-block scale (blocks of 8 padded couplings of a row),
// BF16 hi + lo pairs (streaming kernels, sb_stream_kernels.hpp)
enum : int { kJFp16 = 0, kJBf16 = 1, kJFp32 = 2, kJFp8 = 3, kJFp8Blk = 4, kJBf16x2 = 5 };

// LDS bytes of one batch workgroup of `tpb` threads with `tail_words` of
// staged couplings: two position buffers (slots plus one pad word per lane
// of a wave), the per-wave reduction area, the item word, the tails.
constexpr size_t batch_lds_bytes(int tpb, int tail_words) {
    return sizeof(float) * 2 * (static_cast<size_t>(tpb) * kBatchSPT + 64) +
           sizeof(double) * static_cast<size_t>(tpb / 64) * 64 + 16 +
           sizeof(uint32_t) * static_cast<size_t>(tail_words);
}

struct BatchEvent {
    int n, nnz;
    int row_off;                 // offset into per-spin arrays (a, h, perm, best_T, T rows)
    int rp_off;                  // offset into row_ptr (row_off + event index)
    int nz_off;                  // offset into col, b, J16
    int lg_agents;               // log2 of the agents one work item holds
    int event_id;                // Philox counter word 2
    float c0_scale;              // c0 of the event = (fixed or auto c0) * c0_scale
};

struct BatchArgs {
    int E, M, K, ckpt_every, n_ckpt;
    int n_items, item_begin;     // this launch's items: [item_begin, item_begin + n_items)
    int grid, tail_cap;          // persistent workgroups; LDS words for staged couplings
    uint32_t seed_lo, seed_hi;
    float dt, dta0;
    double c0_fixed;             // > 0: fixed c0 for every event
    const BatchEvent *ev;        // [E]
    const int *item_event;       // [n_items], decreasing cost
    const int *item_agent0;      // [n_items]
    const int *row_ptr;          // [sum (n + 1)] per-event row pointers (local)
    const int *col;              // [sum nnz] per-event spin ids (local)
    const double *a;             // [sum n]
    const double *b;             // [sum nnz]
    uint16_t *J16;               // [sum nnz] 16-bit couplings (prep output)
    float *h;                    // [sum n]
    float *c0;                   // [E]
    double *offset;              // [E] Ising offset C
    int *perm;                   // [sum n] spin order per event
    const float *sched;          // [K]
    int *counter;                // this launch's work queue counter
    double *etrace;              // [E * n_ckpt * M]
    double *energy;              // [E * M] final O(T)
    double *trace;               // [E * n_ckpt] best so far, or null
    double *best_energy;         // [E]
    int *best_agent;             // [E]
    int8_t *T;                   // [sum n * M] final T per agent
    float *x_out;                // [sum n * M] final positions, or null
    int8_t *best_T;              // [sum n]
    long long *ckpt_clock;       // [E * (n_ckpt + 1) * M] device wall clock at each
                                 //   agent's item start and checkpoints, or null
    const double *target;        // [E] or null: stop an event's work at the first
                                 //   checkpoint where an agent reaches O(T) <= target
    int *done;                   // [E] events whose target was reached (target mode)
    // events run as gangs of row bands (sb_batch_gang.hip)
    int gang_items;              // (gang, band) items, gang-major
    const int *gitem_gang;       // [gang_items]
    const int *gitem_band;       // [gang_items]
    const struct GangDesc *gangs;
    float *xg;                   // per gang: two position buffers of n floats
    int *arrive;                 // per gang: bands arrived at its barriers
    double *gpart;               // per gang: [bands][n_ckpt + 1] partial energies
    long long *gclock;           // per gang: [bands][n_ckpt + 1] wall-clock stamps
    int *gang_fault;             // set when a bounded gang wait ran out
    int *gang_counter;           // work queue of the gang launch
};

// One gang: the `bands` row bands of one (event, agent), each of at most
// `rows` consecutive spins, run by as many workgroups at once; positions
// cross bands through the gang's global buffers, one barrier per step.
struct GangDesc {
    int e, agent, bands, rows;
    long long x_off;             // offset of the gang's two position buffers in xg
    int part_off;                // offset of its [bands][n_ckpt + 1] in gpart / gclock
};

hipError_t launch_batch_prep(int jprec, const BatchArgs &B, hipStream_t st);
// resets the launch counters (kernels, so the reset can be graph-captured)
hipError_t launch_batch_reset(int *counters, int n, hipStream_t st);
hipError_t launch_batch_steps(int mode, int jprec, int tpb, const BatchArgs &B, hipStream_t st);
// the step kernel of one mode, coupling format and shape, instantiated in
// its own translation unit (sb_batch_mode.hip, built once per triple)
template <int MODE, int JP, int TPB>
hipError_t launch_batch_steps_tu(const BatchArgs &B, hipStream_t st);

hipError_t launch_batch_select(const BatchArgs &B, hipStream_t st);
// the gang launch (persistent grid of `B.grid` 1024-thread workgroups) and
// the reduction of its partial energies and stamps; n_gangs gangs
hipError_t launch_batch_gang(int mode, int jprec, const BatchArgs &B, hipStream_t st);
hipError_t launch_batch_gang_reduce(const BatchArgs &B, int n_gangs, hipStream_t st);
// zeroes n ints (a kernel, so it can be graph-captured)
hipError_t launch_zero_ints(int *p, int n, hipStream_t st);

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
// the register-row step kernel of one mode (one translation unit each)
hipError_t launch_resident_reg_bsb(const ResidentArgs &A, const ResidentShape &S, hipStream_t st);
hipError_t launch_resident_reg_dsb(const ResidentArgs &A, const ResidentShape &S, hipStream_t st);
hipError_t launch_resident_reg_asb(const ResidentArgs &A, const ResidentShape &S, hipStream_t st);
hipError_t launch_energy(int n, int M, const double *a, const int *row_ptr, const int *col,
                         const double *b, const float *x, double *part, double *out,
                         hipStream_t st);
hipError_t launch_select_best(int n, int M, const double *E, const float *x, double *best_e,
                              int *best_m, int8_t *T, hipStream_t st);
hipError_t launch_trace_reduce(int n_ckpt, int M, const double *et, double *trace, hipStream_t st);

}  // namespace sbt
