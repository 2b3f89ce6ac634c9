/*
 * sbtrack.h -- C ABI of the MI355X simulated-bifurcation track-QUBO library.
 *
 * The library implements the method of Okawa, Zeng, Tao, Yung,
 * "Quantum-Annealing-Inspired Algorithms for Track Reconstruction at
 * High-Energy Colliders":
 *   hits -> QUBO over hit triplets   (sections "QUBO Formulation" and
 *                                     "QUBO Generation and Track Finding")
 *   QUBO -> lowest-energy assignment by ballistic / discrete simulated
 *           bifurcation               (section "Simulated Bifurcation")
 * The solver runs entirely in HIP kernels for gfx950 (CDNA4).
 *
 * Conventions for every function:
 *   - the return value is a status: SBT_OK (0) or a negative SBT_E* code;
 *     sbt_last_error() then returns a thread-local message.  No C++
 *     exception crosses this interface.
 *   - inputs are borrowed for the duration of the call; outputs go into
 *     caller-owned buffers, except an sbt_qubo, which the library allocates
 *     and sbt_qubo_free releases.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device allocations on the current device.
 *   - results are deterministic: the same inputs, parameters and seed give
 *     bit-identical outputs on every run.
 */
#ifndef SBTRACK_H
#define SBTRACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBT_OK 0
#define SBT_EINVAL (-1)       /* invalid argument; nothing was written        */
#define SBT_ENOMEM (-2)       /* host or device allocation failed             */
#define SBT_EDEVICE (-3)      /* a HIP runtime call or kernel launch failed   */
#define SBT_EUNSUPPORTED (-4) /* valid request outside what is implemented    */

/* Thread-local description of the last failure on this thread ("" if none). */
const char *sbt_last_error(void);

/* Library version string. */
const char *sbt_version(void);

/* ------------------------------------------------------------------------
 * Hits and QUBO construction (host, FP64)
 * ---------------------------------------------------------------------- */

/* One silicon hit (paper, Dataset section: barrel layers only).  Lengths in
 * mm.  layer counts outward from 0; doublets join layers L and L+1. */
typedef struct {
    int64_t hit_id; /* caller's id; triplets are ordered by these ids      */
    int32_t layer;
    int32_t pad;    /* ignored                                            */
    double x, y, z;
} sbt_hit;

/* Construction parameters.  sbt_build_params_default() fills the values
 * used throughout: doublet window |dphi| < 0.1 rad; Eq. 16: |kappa| <=
 * 8e-4 mm^-1, dtheta <= 0.1 rad, holes <= 1; Eq. 17: |dkappa| <= 1e-4,
 * S > 0.2; five-hit rule with min(5, layers); Eq. 15 alpha, beta, gamma,
 * lambda = 0.5, 0.2, 1.0, 0.5 (d0, z0 in mm). */
typedef struct {
    double dphi_tan;       /* tan of the doublet azimuth window             */
    double z0_max;         /* doublet |z0| cut in mm; <= 0 disables it      */
    double curv_max;       /* Eq. 16 curvature bound, mm^-1                 */
    double dtheta_tan;     /* Eq. 16: tan of the r-z angle bound            */
    double dcurv_max;      /* Eq. 17 curvature-difference bound, mm^-1      */
    double s_min;          /* Eq. 17 lower bound on S_ij (exclusive)        */
    int32_t max_holes;     /* Eq. 16                                        */
    int32_t min_track_hits;/* five-hit rule; -1 = min(5, number of layers); */
                           /* values above 5 are SBT_EUNSUPPORTED           */
    double alpha, beta, gamma_, lambda_; /* Eq. 15                          */
} sbt_build_params;

void sbt_build_params_default(sbt_build_params *p);

/* A QUBO O(a, b, T) = sum_i a_i T_i + sum_{j<i} b_ij T_i T_j (Eq. 13) over
 * triplets, with b symmetric (both triangles stored, zero diagonal) in CSR
 * with ascending columns.  Host memory owned by the library. */
typedef struct {
    int32_t n;          /* number of triplets (QUBO variables)                */
    int64_t nnz;        /* stored entries of b                                 */
    double *a;          /* [n]     bias weights, Eq. 15                        */
    int64_t *row_ptr;   /* [n+1]                                               */
    int32_t *col;       /* [nnz]                                               */
    double *b;          /* [nnz]   +1 conflict, -S_ij quadruplet (Eq. 14)      */
    int64_t *trip_hits; /* [3n]    hit ids of triplet i, layer order           */
} sbt_qubo;

/* Build the QUBO of Eq. 13 from hits (paper: "QUBO Formulation", "QUBO
 * Generation and Track Finding"): adjacent-layer doublets, triplets cut by
 * Eq. 16, quadruplets cut by Eq. 17 and the five-hit rule, triplets outside
 * every kept quadruplet dropped, triplets indexed in ascending
 * (id1, id2, id3) order, a_i from Eq. 15 and b_ij from Eq. 13/14.
 *   hits    host [n_hits]; any order; hit ids must be distinct
 *   p       host; NULL = defaults
 *   out     receives a library-owned QUBO (n may be 0); free with sbt_qubo_free
 * Errors: SBT_EINVAL for n_hits < 0, non-finite coordinates, negative layers
 * or duplicate ids. */
int sbt_build_qubo(const sbt_hit *hits, int64_t n_hits, const sbt_build_params *p,
                   sbt_qubo **out);
void sbt_qubo_free(sbt_qubo *q);

/* The same construction as sbt_build_qubo computed on the GPU (host hits
 * in, library-owned host QUBO out).  The host sorts the hits and lists each
 * layer by azimuth; doublets, triplets, quadruplets, the five-hit rule,
 * biases, conflicts and the CSR assembly run on the device with the host
 * builder's fixed-order FP64 expressions, so n, row_ptr, col and trip_hits
 * equal sbt_build_qubo's; a and b can differ in the last place where exp
 * (Eq. 15) or atan2 (Eq. 14) enter.
 *   elapsed_s  out or NULL: device time of the construction (HIP events)
 * Errors: as sbt_build_qubo, plus SBT_EDEVICE for HIP failures and
 * SBT_EUNSUPPORTED beyond 32-bit counts. */
int sbt_build_qubo_gpu(const sbt_hit *hits, int64_t n_hits, const sbt_build_params *p,
                       sbt_qubo **out, double *elapsed_s);

/* ------------------------------------------------------------------------
 * Simulated annealing on the CPU (the comparator of section "Simulated
 * Annealing": single-spin moves accepted by the Metropolis rule while the
 * temperature falls)
 * ---------------------------------------------------------------------- */

typedef struct {
    int32_t shots;      /* independent runs >= 1 (each from T = 0)           */
    int32_t sweeps;     /* passes over the spins in index order >= 1         */
    double beta_hot;    /* first inverse temperature; <= 0: ln 2 / the       */
                        /* largest possible energy change                    */
    double beta_cold;   /* last one (geometric in between); <= 0: ln 100 /   */
                        /* the smallest nonzero |a_i| or |b_ij|              */
    uint64_t seed;      /* shot s uses its own stream from (seed, s)         */
    int32_t threads;    /* host threads; 0 = all hardware threads            */
    int32_t reserved;   /* 0                                                 */
} sbt_anneal_params;

/* shots = 50, sweeps = 1000, automatic temperatures, seed 0, all threads. */
void sbt_anneal_params_default(sbt_anneal_params *p);

/* Anneal the QUBO in host memory; O(T) (Eq. 13, FP64) of every shot's
 * final T, the best (lowest shot index on ties) returned.
 *   T_best       caller [n]      energy  out: O(T_best)
 *   shot_energy  caller [shots] or NULL   elapsed_s  out or NULL: wall time
 * Errors: SBT_EINVAL for a malformed QUBO or parameters. */
int sbt_anneal_cpu(const sbt_qubo *q, const sbt_anneal_params *p, int8_t *T_best,
                   double *energy, double *shot_energy, double *elapsed_s);

/* Spin order for the solver's caches (a relabelling only; the section
 * "QUBO formulation" fixes the problem, not its index order): triplets
 * sorted by the azimuth of their middle hit, then its z, then index.  The
 * azimuth is compared through the exact monotone key 1 - x/(|x|+|y|) for
 * y >= 0 and 3 + x/(|x|+|y|) for y < 0 (0 for x = y = 0).
 *   q     QUBO from sbt_build_qubo (its trip_hits name hit ids)
 *   hits  the hits it was built from, any order
 *   perm  caller [n]: perm[k] = original index of the triplet placed at k
 * Errors: SBT_EINVAL for NULL arrays or a triplet naming an absent hit. */
int sbt_phi_order(const sbt_qubo *q, const sbt_hit *hits, int64_t n_hits, int32_t *perm);

/* The same QUBO with spins relabelled: row/column k of the result is
 * row/column perm[k] of q (columns ascending again), a and trip_hits
 * follow.  O(T') of the result equals O(T) of q for T'[k] = T[perm[k]].
 * Library-owned result; free with sbt_qubo_free.
 * Errors: SBT_EINVAL if perm is not a permutation of 0..n-1. */
int sbt_qubo_permute(const sbt_qubo *q, const int32_t *perm, sbt_qubo **out);

/* Exact FP64 value of Eq. 13 for a binary assignment (host, compensated
 * summation, rows in order, pairs j > i).  T host [n] of 0/1. */
int sbt_energy(const sbt_qubo *q, const int8_t *T, double *energy);

/* ------------------------------------------------------------------------
 * Simulated bifurcation (HIP)
 * ---------------------------------------------------------------------- */

/* bSB (Eq. 5-8), dSB (Eq. 9-12), aSB (Eq. 1-4: the quartic potential, no
 * walls; every kernel but the matrix-core dSB step runs it, and its
 * explicit steps need a dt small enough for the cubic force -- the paper
 * defines it but reports bSB and dSB). */
typedef enum { SBT_BSB = 0, SBT_DSB = 1, SBT_ASB = 2 } sbt_mode;

/* Which step kernel runs.  AUTO picks by problem shape. */
typedef enum {
    SBT_KERNEL_AUTO = 0,
    SBT_KERNEL_RESIDENT = 1, /* one launch for all steps; a workgroup owns
                                whole agents, positions live in LDS        */
    SBT_KERNEL_STREAM = 2,   /* one launch per step; state streams through
                                HBM, lanes are agents.  bSB / aSB with
                                agents a multiple of 4 above 64: a wave
                                takes four consecutive rows and gathers each
                                distinct neighbour of the four once (lists
                                built on the GPU once per solve; the
                                workspace grows by about 20 bytes per
                                coupling); otherwise one row per wave      */
    SBT_KERNEL_STREAM_TILE = 3, /* bSB / aSB: the streaming step with rows in
                                planned tiles -- runs of consecutive rows
                                (within blocks of 32) whose column union
                                fits 192 columns -- whose neighbours'
                                positions (the union x 64 agents) are staged
                                in LDS each step; a row longer than that is
                                read from global memory.  The same
                                arithmetic, bit-identical results; every
                                streaming coupling form.  Planned once per
                                solve on the GPU; the workspace grows by
                                6 bytes per padded coupling.  Only on
                                request (AUTO never picks it)            */
    SBT_KERNEL_STREAM_ROWS = 4, /* the streaming step one row per wave for
                                every mode and agent count (what
                                SBT_KERNEL_STREAM runs where it takes no
                                quads); the same arithmetic as the quad
                                step, bit-identical results             */
    SBT_KERNEL_STREAM_MFMA = 5 /* dSB on the matrix cores (Eq. 10 as a
                                product of a dense coupling block and
                                +-1 signs): blocks of 16 consecutive rows
                                list their distinct columns, padded to
                                steps of 32, with the couplings as dense
                                operand tiles; FP8 (per-row scale: the
                                codes are the operand, the scale applies
                                to the row's sum), BF16X2 (hi and lo
                                operands), FP32 (split exactly into
                                three BF16 operands), FP8_BLOCK (each
                                coupling's FP32 value split the same
                                way), BF16 or FP16 (one operand); bSB
                                and aSB give SBT_EUNSUPPORTED.  The products are
                                exact; the FP32 sums are added in the
                                instruction's order, so results differ
                                from the CSR step by rounding.  Planned
                                once per solve on the GPU; the workspace
                                grows by about (nnz / 32 + n / 16) x 640
                                bytes (FP8), x 1152 (BF16, FP16), x 2176
                                (BF16X2) or x 3200 (FP32, FP8_BLOCK),
                                plus x
                                and y in the step's own tiles (rows
                                padded to 16, agents to 128).  AUTO
                                picks it for dSB from n x agents >= 2^23
                                on                                       */
} sbt_kernel;

/* Storage precision of the couplings J.  The paper fixes no number format
 * (section "Simulated Bifurcation" states the dynamics only); the narrow
 * forms are this library's: only J is stored narrower, accumulation is FP32
 * and energies are FP64 of the exact QUBO throughout.
 * FP8 is OCP e4m3 with one FP32 scale per row, max_j |J_ij| / 448;
 * FP8_BLOCK the same with one FP32 scale per block of 8 consecutive stored
 * couplings of a row (the last block of a row may be shorter);
 * BF16X2 stores each FP32 coupling as a BF16 pair hi = bf16(J),
 * lo = bf16(J - hi), used as hi + lo (16 significant bits).
 * FP16 and BF16 (J rounded once) are the batch functions' forms, and for
 * dSB the matrix-core streaming step's; FP8, FP8_BLOCK and BF16X2 run on
 * the streaming kernels. */
typedef enum {
    SBT_PREC_FP32 = 0,
    SBT_PREC_FP16 = 1,
    SBT_PREC_BF16 = 2,
    SBT_PREC_FP8 = 3,
    SBT_PREC_FP8_BLOCK = 4,
    SBT_PREC_BF16X2 = 5
} sbt_precision;

/* Solver parameters (section "Simulated Bifurcation" and Results: a0 = dt = 1,
 * fixed c0).  sbt_solve_params_default() fills a0 = dt = 1, c0 = auto,
 * agents = 32, steps = 2000, seed = 0, event = 0, kernel = AUTO,
 * energy_every = 0, tpb = 0, precision = FP32. */
typedef struct {
    double a0;            /* a0 > 0                                          */
    double dt;            /* time step > 0                                   */
    double c0;            /* coupling scale; <= 0 or NaN: 0.5/(sqrt(N) sd(J)) */
                          /* with sd the population std of all N^2 entries  */
    int32_t agents;       /* independent shots M >= 1                        */
    int32_t steps;        /* symplectic-Euler steps K >= 1                   */
    uint64_t seed;        /* Philox key                                      */
    int32_t event;        /* Philox counter word 2 (batch position)          */
    int32_t kernel;       /* sbt_kernel                                      */
    int32_t energy_every; /* > 0: record the best O(T) every that many steps */
    int32_t tpb;          /* resident kernel threads per workgroup (64, 256,  */
                          /* 512, 1024); 0 = chosen from the shape           */
    int32_t precision;    /* sbt_precision of J for sbt_solve/sbt_solve_dev: */
                          /* FP32 (any kernel) or FP8, FP8_BLOCK, BF16X2     */
                          /* (stream kernel only); the batch functions take  */
                          /* theirs as an argument                           */
    int32_t reserved;     /* must be 0                                       */
} sbt_solve_params;

void sbt_solve_params_default(sbt_solve_params *p);

/* Host-memory result of sbt_solve. */
typedef struct {
    int8_t *T;            /* caller [n] or NULL: best agent's T = (1+sgn x)/2 */
    double *agent_energy; /* caller [agents] or NULL: O(T) of every agent     */
    double *trace;        /* caller [steps/energy_every] or NULL              */
    float *x_final;       /* caller [n*agents] or NULL: final positions,      */
    float *y_final;       /*   spin-major, agents contiguous (index i*M + m)  */
    double energy;        /* out: O(T) of the best agent (Eq. 13, FP64)       */
    double ising_offset;  /* out: C with O(T) = E_ising(s) + C                */
    double c0;            /* out: the c0 used                                 */
    int32_t best_agent;   /* out: argmin of O over agents, lowest on ties     */
    int32_t kernel_used;  /* out: sbt_kernel that ran                         */
    double elapsed_s;     /* out: device time of the solve (HIP events)       */
    double *agent_trace;  /* caller [(steps/energy_every) * agents] or NULL:  */
                          /*   O(T) of every agent at every checkpoint        */
                          /*   (checkpoint-major; checkpoint c is the state   */
                          /*   after (c+1) * energy_every steps)              */
    int32_t trace_len;    /* out: checkpoints written to trace and            */
                          /*   agent_trace, steps / energy_every (0 without)  */
} sbt_result;

/* Solve one QUBO held in host memory: upload, run every step on the GPU,
 * download.  Allocates and frees its device memory internally.
 * Integration (Eq. 5-8 for BSB, Eq. 9-12 for DSB), for k = 0..K-1:
 *   a_k = a0 k / K
 *   F   = J x + h            (BSB)   or   J sgn(x) + h   (DSB), sgn(0) = +1
 *   y  += dt (c0 F - (a0 - a_k) x);   x += dt a0 y
 *   |x| > 1  ->  x = sgn(x), y = 0
 * with J = -b/4, h = -(a/2 + rowsum(b)/4), starting from the Philox4x32-10
 * draw x0, y0 in [-1/8, 1/8) (counter = (spin, agent, event, 0),
 * key = seed).  Readout T = (1 + sgn x)/2 per agent; energies are FP64.
 * Errors: SBT_EINVAL for an empty or malformed QUBO (non-finite values,
 * unsorted or out-of-range columns, diagonal entries, asymmetric b) or
 * invalid parameters; SBT_EDEVICE for HIP failures. */
int sbt_solve(const sbt_qubo *q, sbt_mode mode, const sbt_solve_params *p,
              sbt_result *out);

/* Device-resident form used when the QUBO already lives in HBM (the path
 * the benchmark times).  All pointers are device pointers; nothing is
 * allocated: scratch comes from `workspace`.  Contents of the QUBO are not
 * validated (sbt_solve validates host data); sizes and parameters are. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const double *a;       /* device [n]                                       */
    const int32_t *row_ptr;/* device [n+1], row_ptr[0] = 0, row_ptr[n] = nnz  */
    const int32_t *col;    /* device [nnz], ascending per row, no diagonal     */
    const double *b;       /* device [nnz], symmetric                          */
} sbt_dev_qubo;

typedef struct {
    int8_t *T;            /* device [n]: best agent's assignment              */
    double *agent_energy; /* device [agents]                                  */
    double *best_energy;  /* device [1]                                       */
    int32_t *best_agent;  /* device [1]                                       */
    double *scalars;      /* device [4] or NULL: c0, C, sum J, sum J^2        */
    float *x_final;       /* device [n*agents] or NULL                        */
    float *y_final;       /* device [n*agents] or NULL                        */
    double *trace;        /* device [steps/energy_every] or NULL              */
    void *step_begin;     /* hipEvent_t or NULL: recorded on the stream just  */
    void *step_end;       /*   before the first and after the last SB-step    */
                          /*   kernel, to time the step phase                 */
    double *agent_trace;  /* device [(steps/energy_every) * agents] or NULL:  */
                          /*   O(T) of every agent at every checkpoint,       */
                          /*   checkpoint-major (see sbt_result)              */
} sbt_dev_result;

/* Bytes of device workspace sbt_solve_dev needs for this shape; 0 on
 * invalid arguments (message in sbt_last_error). */
size_t sbt_workspace_bytes(int32_t n, int64_t nnz, sbt_mode mode,
                           const sbt_solve_params *p);

/* Which kernel AUTO selects for this shape (sbt_kernel), or a negative
 * status. */
int sbt_select_kernel(int32_t n, int64_t nnz, int32_t max_row_nnz, sbt_mode mode,
                      const sbt_solve_params *p);

/* Run a solve on device data, enqueued on `stream` (a hipStream_t; NULL =
 * the default stream).  Returns after enqueueing; results are ready when
 * the stream reaches this point.  `max_row_nnz` is the largest row length
 * of b (used to pick and size kernels).  Calls that share a workspace must
 * not overlap. */
int sbt_solve_dev(const sbt_dev_qubo *q, int32_t max_row_nnz, sbt_mode mode,
                  const sbt_solve_params *p, void *workspace, size_t workspace_bytes,
                  const sbt_dev_result *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as sbt_solve_dev with no workspace argument.  Its scratch lives in
 * a fixed array of SBT_NOALLOC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends; the call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  Inputs and
 * outputs are the caller's device buffers, as for sbt_solve_dev.
 * All calls on one device share that array and it keeps the last call's
 * contents, so calls that overlap on one device (other streams, other host
 * threads) race: serialise them.
 * Errors: SBT_EINVAL when sbt_workspace_bytes for this shape exceeds
 * SBT_NOALLOC_SCRATCH_BYTES (checked before any device call), otherwise as
 * sbt_solve_dev. */
#define SBT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int sbt_solve_dev_noalloc(const sbt_dev_qubo *q, int32_t max_row_nnz, sbt_mode mode,
                          const sbt_solve_params *p, const sbt_dev_result *out, void *stream);

/* The k lowest agent energies (paper section "Results": the best of the
 * shots, here the best k of them, as the stress workload reports its best
 * 32), on the GPU.  energy: device [agents], FP64 O(T) per agent (e.g.
 * sbt_dev_result.agent_energy); top_energy, top_agent: device [k], written
 * in ascending (energy, agent) order -- ties go to the lower agent, as for
 * best_agent, and NaN energies come after every number.  One workgroup,
 * queued on `stream` (hipStream_t or NULL); allocates nothing.
 * Errors: SBT_EINVAL for NULL pointers, agents < 1 or k outside
 * 1..agents (checked before any device call); SBT_EDEVICE if the launch
 * fails. */
int sbt_top_k_dev(const double *energy, int32_t agents, int32_t k, double *top_energy,
                  int32_t *top_agent, void *stream);

/* ------------------------------------------------------------------------
 * Batches of events (HIP)
 *
 * Many independent events solved together (the paper solves one event at a
 * time; batching only changes the scheduling).  Every event gets `agents`
 * agents and `steps` steps of the same form (section "Simulated
 * Bifurcation"), event e drawing its start with Philox counter word
 * p->event + e.  All events run in one persistent kernel: work items are
 * (event, group of agents) taken from a queue in decreasing-cost order, each
 * workgroup holding all positions of its agents on chip.  The couplings are
 * held in 16 bits (the reduced-precision form); accumulation is FP32 and
 * energies are FP64 of the returned spins.
 * ---------------------------------------------------------------------- */

/* Events concatenated in device memory. */
typedef struct {
    int32_t n_events;
    const int32_t *n;        /* host [E]: variables of each event (>= 1; above   */
                             /*   9216 as gangs of row bands, at most 9216 x the  */
                             /*   device's CU count)                              */
    const int64_t *nnz;      /* host [E]: stored couplings of each event          */
    const double *a;         /* device [sum n]                                     */
    const int32_t *row_ptr;  /* device [sum (n + 1)]: each event's own CSR row    */
                             /*   pointers, starting at 0                          */
    const int32_t *col;      /* device [sum nnz]: columns local to the event      */
    const double *b;         /* device [sum nnz]: symmetric, ascending columns    */
    const double *target;    /* device [E] or NULL.  Target mode (time-to-target: */
                             /*   stop at the goal, as a solve run for time-to-   */
                             /*   solution would): event e's work stops at the    */
                             /*   first checkpoint (energy_every > 0 required)    */
                             /*   where one of its agents reaches O(T) <=         */
                             /*   target[e] (an event run as gangs of row bands:  */
                             /*   each agent's gang stops on its own energy); its */
                             /*   agents keep the state reached (results are of  */
                             /*   that state), the checkpoints not reached read   */
                             /*   NaN in agent_trace.  The items of one event     */
                             /*   stop through a shared flag, so at which         */
                             /*   checkpoint each stops depends on timing: a      */
                             /*   target-mode solve is not bit-reproducible       */
} sbt_dev_batch;

typedef struct {
    double *best_energy;     /* device [E]: O(T) of each event's best agent       */
    int32_t *best_agent;     /* device [E]                                         */
    int8_t *best_T;          /* device [sum n]: best agent's T, events concatenated */
    double *agent_energy;    /* device [E * agents] or NULL                        */
    double *offset;          /* device [E] or NULL: Ising offsets C                */
    double *trace;           /* device [E * (steps / energy_every)] or NULL:      */
                             /*   best-so-far O(T) per checkpoint                  */
    void *step_begin;        /* hipEvent_t or NULL, recorded around the kernel    */
    void *step_end;          /*   that runs every step of every event             */
    int8_t *agent_T;         /* device [sum n * agents] or NULL: every agent's    */
                             /*   final T (event e's block spin-major, agents     */
                             /*   contiguous, starting at agents * sum_{f<e} n_f) */
    float *agent_x;          /* device [sum n * agents] or NULL: final positions, */
                             /*   same layout                                     */
    double *agent_trace;     /* device [E * (steps / energy_every) * agents] or   */
                             /*   NULL: O(T) of every agent at every checkpoint   */
                             /*   (event-major, then checkpoint, then agent)      */
    int64_t *ckpt_clock;     /* device [E * (steps / energy_every + 1) * agents]  */
                             /*   or NULL: device wall-clock ticks (see           */
                             /*   sbt_wall_clock_hz) when each agent's work item  */
                             /*   starts (slot 0) and when its checkpoint c       */
                             /*   energy is known (slot c + 1); for measuring     */
                             /*   time-to-target inside the one batch launch      */
} sbt_dev_batch_result;

/* How a batch is scheduled: which events run on which step-kernel shape
 * and how many agents a work item holds.  Scheduling only: every agent
 * performs the same step arithmetic in the same order under any tuning, so
 * positions and assignments are bit-identical; the FP64 energies are summed
 * in an order that follows the schedule and agree to rounding.
 * Shapes: 1024 threads per workgroup, one workgroup per CU (any n up to
 * 9216), and 512 threads, two workgroups per CU (n up to 4608), each with 9
 * position slots per thread.  The 1024-thread items run first, then the
 * 512-thread items, each as one persistent launch over its own queue. */
typedef struct {
    int32_t split_n;     /* events with n <= split_n (and n <= 4608) run on the */
                         /*   512-thread shape; 0 = every event on 1024 threads */
    int32_t tail_words;  /* LDS words per workgroup for couplings past the     */
                         /*   register capacity of their slot, 0..8192          */
    double fill;         /* an item holds A agents, A the largest power of two */
                         /*   with n A <= fill x (slots of its shape), A <=    */
                         /*   agents and A <= threads; fill in (0, 1]          */
    int32_t band_rows;   /* events with n above this (0 = 9216, the largest    */
                         /*   that one workgroup holds; at most 9216) run as    */
                         /*   gangs of row bands: one gang per agent, bands of  */
                         /*   at most band_rows consecutive spins on as many    */
                         /*   workgroups at once, positions exchanged through   */
                         /*   HBM with one barrier per step                     */
    int32_t from_cache;  /* out of sbt_batch_tuning_lookup: 1 = tuned entry    */
    int32_t reserved;    /* must be 0                                          */
} sbt_batch_tuning;

/* split_n = 0, tail_words = 8192, fill = 1 (what the untuned entry points
 * use). */
void sbt_batch_tuning_default(sbt_batch_tuning *t);

/* The tuning cache key of a batch: mode, precision, agents and a histogram
 * of event sizes (counts of n <= 64, <= 128, ..., <= 16384).  key receives a
 * NUL-terminated string of at most key_len bytes. */
int sbt_batch_tuning_key(const int32_t *n, int32_t n_events, sbt_mode mode, sbt_precision prec,
                         int32_t agents, char *key, size_t key_len);

/* The tuned schedule for a batch from the project's tuning cache (a JSON
 * file written by the tuner, paper_2402_14718_amd/autotune.py; path from
 * the environment variable SBT_BATCH_TUNING_CACHE, else tuning/
 * batch_tuning.json beside the library; read once per process): the entry
 * with this batch's key, else the entry of the same mode, precision and
 * agents whose normalised size histogram is nearest (L1 distance <= 0.25),
 * else the defaults (out->from_cache tells which). */
int sbt_batch_tuning_lookup(const int32_t *n, int32_t n_events, sbt_mode mode,
                            sbt_precision prec, int32_t agents, sbt_batch_tuning *out);

/* Device workspace bytes for a batch of these sizes (0 on invalid input),
 * with the default tuning / with tuning t (NULL = default). */
size_t sbt_batch_workspace_bytes(const int32_t *n, const int64_t *nnz, int32_t n_events,
                                 const sbt_solve_params *p);
size_t sbt_batch_workspace_bytes_tuned(const int32_t *n, const int64_t *nnz, int32_t n_events,
                                       const sbt_solve_params *p, const sbt_batch_tuning *t);

/* Upload the batch's schedule (event descriptors and the ordered work
 * items) into `workspace` on `stream`.  Call once per (batch shape,
 * parameters); sbt_batch_run then only launches kernels and may be captured
 * in a HIP graph.
 *   c0_scale    host [E] or NULL: event e runs with c0 * c0_scale[e] (c0 the
 *               fixed or automatic value of that event); each > 0
 *   same_start  nonzero: every event draws its start with counter word
 *               p->event (a scan of one QUBO); zero: event e uses p->event + e
 * Returns the number of work items (row-band items of gangs included), or a
 * negative status; SBT_EUNSUPPORTED for an event needing more row bands
 * than the device has CUs (the bands of a gang must run at once). */
int sbt_batch_plan(const int32_t *n, const int64_t *nnz, int32_t n_events,
                   const double *c0_scale, int32_t same_start, const sbt_solve_params *p,
                   void *workspace, size_t workspace_bytes, void *stream);
/* The same with tuning t (NULL = default); run the batch with the same t. */
int sbt_batch_plan_tuned(const int32_t *n, const int64_t *nnz, int32_t n_events,
                         const double *c0_scale, int32_t same_start, const sbt_solve_params *p,
                         const sbt_batch_tuning *t, void *workspace, size_t workspace_bytes,
                         void *stream);

/* Solve every event of a planned batch: per-event Ising preparation and
 * spin ordering, all steps of all agents of all events in one persistent
 * kernel, FP64 energies, best agent per event.  `prec` is SBT_PREC_FP16 or
 * SBT_PREC_BF16 (SBT_EUNSUPPORTED otherwise).  Returns after enqueueing. */
int sbt_batch_run(const sbt_dev_batch *batch, sbt_mode mode, sbt_precision prec,
                  const sbt_solve_params *p, void *workspace, size_t workspace_bytes,
                  const sbt_dev_batch_result *out, void *stream);
/* The same with tuning t (NULL = default), which must be the plan's. */
int sbt_batch_run_tuned(const sbt_dev_batch *batch, sbt_mode mode, sbt_precision prec,
                        const sbt_solve_params *p, const sbt_batch_tuning *t, void *workspace,
                        size_t workspace_bytes, const sbt_dev_batch_result *out, void *stream);

/* Tick rate of the device wall clock that sbt_dev_batch_result.ckpt_clock
 * reads (a constant-rate counter, independent of the shader clock), for
 * the current device. */
int sbt_wall_clock_hz(double *hz);

/* Host-memory results of sbt_solve_batch. */
typedef struct {
    double *energy;          /* caller [E]: best O(T) per event                    */
    int32_t *best_agent;     /* caller [E]                                         */
    int8_t *T;               /* caller [sum n] or NULL: best T, events concatenated */
    double *agent_energy;    /* caller [E * agents] or NULL                        */
    double *trace;           /* caller [E * (steps / energy_every)] or NULL        */
    double elapsed_s;        /* out: device time of plan + run                     */
    double *agent_trace;     /* caller [E * (steps / energy_every) * agents] or    */
                             /*   NULL: as sbt_dev_batch_result.agent_trace        */
} sbt_batch_result;

/* Host convenience: validate and upload the QUBOs, plan, run, download,
 * with the tuned schedule from sbt_batch_tuning_lookup. */
int sbt_solve_batch(const sbt_qubo *const *qs, int32_t n_events, sbt_mode mode,
                    sbt_precision prec, const sbt_solve_params *p, sbt_batch_result *out);

/* Automatic c0 scan (Results: c0 fixed or found by a scan).  Solves the one
 * QUBO q once per factor in a single batch, copy k with c0 * factors[k]
 * (c0 = p->c0 if > 0, else the automatic value), every copy from the same
 * Philox start (counter word p->event).
 *   energy       caller [n_factors]: best FP64 O(T) per factor
 *   best_agent   caller [n_factors]
 *   best_factor  out: index of the lowest energy (lowest index on ties)
 * Errors: as sbt_solve_batch; SBT_EINVAL for a factor that is not finite
 * and > 0. */
int sbt_c0_scan(const sbt_qubo *q, sbt_mode mode, sbt_precision prec, const sbt_solve_params *p,
                const double *factors, int32_t n_factors, double *energy, int32_t *best_agent,
                int32_t *best_factor);

#ifdef __cplusplus
}
#endif

#endif /* SBTRACK_H */
