// Batched SB over many events in one persistent kernel (gfx950).
//
// Paper section "Simulated Bifurcation" (bSB Eq. 5-8, dSB Eq. 9-12) applied
// to a batch of independent events (the paper solves one event at a time;
// batching is this library's scheduling, not a change of the method).
//
// Work items are (event, group of A agents) with A a power of two chosen so
// that n_event * A fills one workgroup's slots; items are ordered by
// decreasing cost and handed out by an atomic counter to a persistent grid.
// Two workgroup shapes exist (the tuner decides which events use which):
// 1024 threads, one workgroup per CU, and 512 threads, two per CU (each
// workgroup's barrier stalls overlap the other's work); both hold 9 slots
// per thread within 128 VGPRs.  Inside an item the structure is the
// register-row resident kernel: positions of the A agents in LDS
// (spin-major, agent-minor: index i*A + a), momenta and couplings in
// VGPRs.  Couplings are stored in 16 bits (FP16 or BF16, the reduced
// precision form) next to a full LDS byte address; accumulation is FP32 and
// energies FP64.
//
// Slot s of thread t is position j = s*TPB + t of the item, spin rank
// q = j / A in decreasing-row-length order, agent a = j % A (so a thread's
// slots all belong to agent t % A).  Register capacity per slot follows the
// row-length profile by rank: slot 0 holds the longest rows.
//
// This header holds the step kernel; sb_batch_mode.hip instantiates it for
// one (mode, coupling format) per build of that file (in parallel),
// sb_batch.hip holds the per-event preparation and the best-agent selection.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <type_traits>

#include "sb_device.hpp"
#include "sb_kernels.hpp"

namespace sbt {

namespace {

constexpr int kS = kBatchSPT;     // slots per thread
// couplings held in registers per slot (rank profile); rows beyond a
// slot's capacity continue from global memory
constexpr int kCap[kS] = {16, 8, 5, 4, 3, 2, 2, 2, 1};

// A held coupling is one VGPR: LDS byte address of the neighbour in the
// first position buffer in the low 16 bits, the 16-bit coupling in the high
// 16 bits.  FP16 converts
// inside the multiply-add (v_fma_mix); BF16 is the upper half of an FP32.
template <int JP>
__device__ __forceinline__ float packed_j(uint32_t cp) {
    if constexpr (JP == kJFp16) {
        return static_cast<float>(__ushort_as_half(static_cast<uint16_t>(cp >> 16)));
    } else {
        return __uint_as_float(cp & 0xFFFF0000u);
    }
}

template <int JP>
__device__ __forceinline__ float j16_to_f32(uint16_t bits) {
    return packed_j<JP>(static_cast<uint32_t>(bits) << 16);
}

// LDS words by absolute address (an address-space-3 pointer made from the
// integer): a constant displacement -- which position buffer a step reads
// or writes -- then folds into the instruction's offset field instead of
// costing an add per access.
typedef __attribute__((address_space(3))) float lds_float;
typedef __attribute__((address_space(3))) unsigned char lds_byte;

__device__ __forceinline__ float lds_load(uint32_t addr) {
    return *(const lds_float *)(static_cast<uintptr_t>(addr));
}

__device__ __forceinline__ void lds_store(uint32_t addr, float v) {
    *(lds_float *)(static_cast<uintptr_t>(addr)) = v;
}

// The neighbour a held coupling names, in the buffer at displacement XO.
template <uint32_t XO>
__device__ __forceinline__ float lds_at(uint32_t cp) {
    return lds_load((cp & 0xFFFFu) + XO);
}

// Hides a loop-invariant register from the optimiser (an empty asm that
// "modifies" it) so that values derived from it are recomputed where used
// instead of being hoisted out of the step loop and kept live: the packed
// couplings exist to save registers.  Emits no instruction.  `launder`
// acts on the register in place (once per step on the loop-carried value:
// no copy); `opaque` returns a laundered copy (for uses outside the loop).
__device__ __forceinline__ void launder(uint32_t &v) { asm volatile("" : "+v"(v)); }

__device__ __forceinline__ uint32_t opaque(uint32_t v) {
    launder(v);
    return v;
}

}  // namespace

// Couplings gathered per step for slot S: C0 for slot 0; the slot's capacity
// for the others, or at most 2 when every row past slot 0 of the wave is
// that short (SH).
template <int C0, bool SH>
constexpr int slot_gathers(int S) {
    return S == 0 ? C0 : (SH && kCap[S] > 2 ? 2 : kCap[S]);
}

// Calls f(integral_constant<int, S>) for S = 0 .. kS-1, so per-slot
// capacities are constant expressions and every register array is indexed
// with constants.
template <int S = 0, class F>
__device__ __forceinline__ void for_slots(F &&f) {
    if constexpr (S < kS) {
        f(std::integral_constant<int, S>{});
        for_slots<S + 1>(f);
    }
}

// At least four waves per SIMD for either shape (128 VGPRs): 1024 threads
// are four waves per SIMD by themselves, 512 threads need the hint so that
// two workgroups fit a CU.
template <int MODE, int JP, int TPB>
__global__ __launch_bounds__(TPB, 4) void sb_batch(BatchArgs B) {
    constexpr int kB = TPB;                     // threads per workgroup
    constexpr int kSlots = kB * kS;             // largest n * A of an item
    constexpr int kStride = kSlots + 64;        // position buffer: slots, one pad word per lane
    extern __shared__ __align__(16) unsigned char smem[];
    float *xs = reinterpret_cast<float *>(smem);                     // [2][kStride]
    double *red = reinterpret_cast<double *>(xs + 2 * kStride);     // [waves][64]
    int *item_s = reinterpret_cast<int *>(red + (kB / 64) * 64);
    // couplings past a slot's register capacity, packed like the held ones
    uint32_t *tails = reinterpret_cast<uint32_t *>(item_s + 4);  // [B.tail_cap]
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;

    for (;;) {
        if (t == 0) *item_s = atomicAdd(B.counter, 1);
        __syncthreads();
        const int local = *item_s;
        __syncthreads();
        if (local >= B.n_items) return;
        const int item = B.item_begin + local;
        const int e = B.item_event[item];
        const int agent0 = B.item_agent0[item];
        const BatchEvent E = B.ev[e];
        const int n = E.n, lgA = E.lg_agents, A = 1 << lgA;
        const int a = t & (A - 1);
        const int agent = agent0 + a;
        const bool agent_ok = agent < B.M;
        // when each agent's work starts and reaches each checkpoint (the
        // device's constant-rate wall clock), for time-to-target
        auto stamp = [&](int slot) __attribute__((always_inline)) {
            if (B.ckpt_clock && t < A && agent0 + t < B.M)
                B.ckpt_clock[(static_cast<size_t>(e) * (B.n_ckpt + 1) + slot) * B.M + agent0 + t] =
                    wall_clock64();
        };
        stamp(0);

        float xr[kS], yr[kS], hr[kS];
        // LDS address of the first position buffer (the dynamic LDS base; the
        // launch checks that it is 0, so every packed address fits 16 bits)
        const uint32_t lds0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_byte *)smem));
        // LDS address, in the first position buffer, of the word each slot's
        // position is stored to: lds0 + 4 (i * A + a) for spin i, a pad
        // word past the slots for a lane without a spin
        uint32_t wr[kS];
        auto spin_of = [&](int S) __attribute__((always_inline)) -> int {
            const uint32_t w = opaque(wr[S]) - lds0;
            return w < static_cast<uint32_t>(4 * kSlots) ? static_cast<int>(w >> (lgA + 2)) : -1;
        };
        uint32_t cp0[kCap[0]], cp1[kCap[1]], cp2[kCap[2]], cp3[kCap[3]], cp4[kCap[4]],
            cp5[kCap[5]], cp6[kCap[6]], cp7[kCap[7]], cp8[kCap[8]];
        auto cps = [&](auto sc) __attribute__((always_inline)) -> uint32_t * {
            constexpr int S = decltype(sc)::value;
            if constexpr (S == 0) return cp0;
            else if constexpr (S == 1) return cp1;
            else if constexpr (S == 2) return cp2;
            else if constexpr (S == 3) return cp3;
            else if constexpr (S == 4) return cp4;
            else if constexpr (S == 5) return cp5;
            else if constexpr (S == 6) return cp6;
            else if constexpr (S == 7) return cp7;
            else return cp8;
        };
        int need0 = 0, tail = 0, act = 0, rest = 0;
        // tail lengths of the slots, 4 bits each: slots 0-7 in tp_lo, slot 8
        // in the low bits of tp_hi (whose upper bits get the LDS offset)
        uint32_t tp_lo = 0, tp_hi = 0;
        int tsum = 0, tbig = 0;
        for_slots([&](auto sc) __attribute__((always_inline)) {
            constexpr int S = decltype(sc)::value;
            constexpr int CAP = kCap[S];
            uint32_t *cp = cps(sc);
            const int j = S * kB + t;
            const int q = j >> lgA;
            const int i = (q < n && agent_ok) ? B.perm[E.row_off + q] : -1;
            // a lane without a spin in an active slot updates a zero
            // oscillator into its own pad word, so steps need no branches
            wr[S] = lds0 + 4u * (i >= 0 ? static_cast<uint32_t>(i * A + a)
                                        : static_cast<uint32_t>(kSlots + lane));
            xr[S] = yr[S] = hr[S] = 0.0f;
#pragma unroll
            for (int c = 0; c < CAP; ++c) cp[c] = 0;
            if (i >= 0) {
                const Philox4 r = philox4x32_10(static_cast<uint32_t>(i), static_cast<uint32_t>(agent),
                                                static_cast<uint32_t>(E.event_id), 0u, B.seed_lo,
                                                B.seed_hi);
                xr[S] = philox_word_to_unit(r.v[0]);
                yr[S] = philox_word_to_unit(r.v[1]);
                hr[S] = B.h[E.row_off + i];
                const int p0 = B.row_ptr[E.rp_off + i], p1 = B.row_ptr[E.rp_off + i + 1];
#pragma unroll
                for (int c = 0; c < CAP; ++c) {
                    if (p0 + c < p1)
                        cp[c] = (lds0 + static_cast<uint32_t>((B.col[E.nz_off + p0 + c] * A + a) * 4)) |
                                (static_cast<uint32_t>(B.J16[E.nz_off + p0 + c]) << 16);
                }
                if (S == 0)
                    need0 = p1 - p0;
                else
                    rest = max(rest, min(p1 - p0, CAP));
                tail |= (p1 - p0 > CAP) ? 1 : 0;
                const int tl = max(0, p1 - p0 - CAP);
                tbig |= tl > 15 ? 1 : 0;
                const uint32_t tl4 = static_cast<uint32_t>(min(tl, 15));
                if constexpr (S < 8)
                    tp_lo |= tl4 << (4 * S);
                else
                    tp_hi |= tl4;
                tsum += tl;
                act |= 1 << S;
                xs[i * A + a] = shared_value<MODE>(xr[S]);
            }
        });
        const int cap0 = wave_max_int(need0);
        const int any_tail = wave_max_int(tail);
        // every row past slot 0 in this wave has at most two couplings
        const bool short_rest = wave_max_int(rest) <= 2;
        // tails staged in LDS once per item (offsets by a block scan); an
        // item whose tails do not fit, or hold more than 15 couplings for
        // one row, reads them from global memory
        int t_total = 0, big_total = 0;
        const int t_base = block_exclusive_scan(tsum, reinterpret_cast<int *>(red), t_total);
        (void)block_exclusive_scan(tbig, reinterpret_cast<int *>(red), big_total);
        const bool lds_tails = t_total <= B.tail_cap && big_total == 0;
        if (lds_tails && tsum > 0) {
            int o = t_base;
            for_slots([&](auto sc) __attribute__((always_inline)) {
                constexpr int S = decltype(sc)::value;
                const int i = spin_of(S);
                if (i >= 0) {
                    const int p0 = B.row_ptr[E.rp_off + i] + kCap[S], p1 = B.row_ptr[E.rp_off + i + 1];
                    for (int p = p0; p < p1; ++p)
                        tails[o++] = (lds0 + static_cast<uint32_t>((B.col[E.nz_off + p] * A + a) * 4)) |
                                     (static_cast<uint32_t>(B.J16[E.nz_off + p]) << 16);
                }
            });
        }
        tp_hi |= lds_tails ? static_cast<uint32_t>(t_base) << 4 : 0u;
        int act_w = act;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) act_w |= __shfl_xor(act_w, off, 64);
        act_w = __builtin_amdgcn_readfirstlane(act_w);
        const int n_act = 32 - __builtin_clz(act_w | 1);  // active slots form a prefix
        __syncthreads();

        const float c0 = B.c0[e];
        const float dt = B.dt, dta0 = B.dta0;
        int ck = 0;

        // per-agent FP64 energy of the current state (Eq. 13); the total of
        // agent t is returned in threads t < A
        auto agent_energy = [&](const float *xv) __attribute__((always_inline)) -> double {
            double v = 0.0;
            for_slots([&](auto sc) __attribute__((always_inline)) {
                constexpr int S = decltype(sc)::value;
                const int i = spin_of(S);
                if (i >= 0 && xr[S] >= 0.0f) {
                    double er = B.a[E.row_off + i];
                    const int p0 = B.row_ptr[E.rp_off + i], p1 = B.row_ptr[E.rp_off + i + 1];
                    for (int p = p0; p < p1; ++p) {
                        const int c = B.col[E.nz_off + p];
                        if (c > i && xv[c * A + a] >= 0.0f) er += B.b[E.nz_off + p];
                    }
                    v += er;
                }
            });
            // lanes with equal t % A hold the same agent
            for (int off = 32; off >= A; off >>= 1) v += __shfl_xor(v, off, 64);
            red[wave * 64 + lane] = v;
            __syncthreads();
            // agent t: lane t of every wave when A <= 64; otherwise lane
            // t % 64 of the waves whose first agent is t rounded down to 64
            double tot = 0.0;
            if (t < A) {
                for (int w = 0; w < kB / 64; ++w) {
                    if (A <= 64)
                        tot += red[w * 64 + t];
                    else if (((w * 64) & (A - 1)) == (t & ~63))
                        tot += red[w * 64 + (t & 63)];
                }
            }
            __syncthreads();
            return tot;
        };

        // The step loop, specialised per wave on its active slots (NA, a
        // prefix) and slot 0's gather count (C0), chosen once per item: a
        // step runs straight through -- gathers, FMAs in CSR order, update,
        // LDS store, barrier -- with rows longer than a slot's capacity
        // (rare) continuing from global memory out of line.  Every variant
        // meets the same barriers.
        // SH: slots past 0 gather min(capacity, 2) couplings (the entries
        // beyond are zero padding in such a wave)
        int k_done = B.K;  // steps taken (fewer when a target stops the event)
        auto run = [&](auto nac, auto c0c, auto shc) __attribute__((always_inline)) {
            constexpr int NA = decltype(nac)::value;
            constexpr int C0 = decltype(c0c)::value;
            constexpr bool SH = decltype(shc)::value;
            auto step = [&](auto bufc, int k) __attribute__((always_inline)) {
                constexpr int BUF = decltype(bufc)::value;
                constexpr uint32_t XO = BUF * kStride * 4;        // buffer read
                constexpr uint32_t XN = (BUF ^ 1) * kStride * 4;  // buffer written
                const unsigned char *xc = smem + XO;
                const float g = B.sched[k];
                float acc[kS];
                for_slots([&](auto sc) __attribute__((always_inline)) {
                    constexpr int S = decltype(sc)::value;
                    if constexpr (S < NA) {
                        acc[S] = hr[S];
                        uint32_t *cp = cps(sc);
                        constexpr int CAP = slot_gathers<C0, SH>(S);
#pragma unroll
                        for (int c = 0; c < CAP; ++c) launder(cp[c]);
                        launder(wr[S]);
                    }
                });
                // slot 0 first; the other slots' gathers are issued after
                // slot 0 has been summed, which bounds the registers in flight
                {
                    float v0[C0];
                    uint32_t w0[C0];
#pragma unroll
                    for (int c = 0; c < C0; ++c) w0[c] = cp0[c];
#pragma unroll
                    for (int c = 0; c < C0; ++c) v0[c] = lds_at<XO>(w0[c]);
#pragma unroll
                    for (int c = 0; c < C0; ++c) acc[0] = __builtin_fmaf(packed_j<JP>(w0[c]), v0[c], acc[0]);
                }
                float v1[kCap[1]], v2[kCap[2]], v3[kCap[3]], v4[kCap[4]], v5[kCap[5]], v6[kCap[6]],
                    v7[kCap[7]], v8[kCap[8]];
                auto vs = [&](auto sc) __attribute__((always_inline)) -> float * {
                    constexpr int S = decltype(sc)::value;
                    if constexpr (S == 1) return v1;
                    else if constexpr (S == 2) return v2;
                    else if constexpr (S == 3) return v3;
                    else if constexpr (S == 4) return v4;
                    else if constexpr (S == 5) return v5;
                    else if constexpr (S == 6) return v6;
                    else if constexpr (S == 7) return v7;
                    else return v8;
                };
                for_slots([&](auto sc) __attribute__((always_inline)) {
                    constexpr int S = decltype(sc)::value;
                    if constexpr (S > 0 && S < NA) {
                        float *v = vs(sc);
                        const uint32_t *cp = cps(sc);
#pragma unroll
                        for (int c = 0; c < slot_gathers<C0, SH>(S); ++c) v[c] = lds_at<XO>(cp[c]);
                    }
                });
                for_slots([&](auto sc) __attribute__((always_inline)) {
                    constexpr int S = decltype(sc)::value;
                    if constexpr (S > 0 && S < NA) {
                        const float *v = vs(sc);
                        const uint32_t *cp = cps(sc);
#pragma unroll
                        for (int c = 0; c < slot_gathers<C0, SH>(S); ++c)
                            acc[S] = __builtin_fmaf(packed_j<JP>(cp[c]), v[c], acc[S]);
                    }
                });
                if (__builtin_expect(any_tail, 0) && lds_tails) {
                    // CSR order within each slot's row, after the held couplings
                    int o = static_cast<int>(tp_hi >> 4);
                    for_slots([&](auto sc) __attribute__((always_inline)) {
                        constexpr int S = decltype(sc)::value;
                        if constexpr (S < NA) {
                            const int len = static_cast<int>((S < 8 ? tp_lo >> (4 * (S & 7)) : tp_hi) & 15u);
                            for (int u = 0; u < len; ++u) {
                                const uint32_t w = tails[o + u];
                                acc[S] = __builtin_fmaf(packed_j<JP>(w), lds_at<XO>(w), acc[S]);
                            }
                            o += len;
                        }
                    });
                } else if (__builtin_expect(any_tail, 0)) {
                    const float *xcf = reinterpret_cast<const float *>(xc);
                    for_slots([&](auto sc) __attribute__((always_inline)) {
                        constexpr int S = decltype(sc)::value;
                        if constexpr (S < NA) {
                            const int i = spin_of(S);
                            if (i >= 0) {
                                const int p1 = B.row_ptr[E.rp_off + i + 1];
                                for (int p = B.row_ptr[E.rp_off + i] + kCap[S]; p < p1; ++p)
                                    acc[S] = __builtin_fmaf(j16_to_f32<JP>(B.J16[E.nz_off + p]),
                                                            xcf[B.col[E.nz_off + p] * A + a], acc[S]);
                            }
                        }
                    });
                }
                for_slots([&](auto sc) __attribute__((always_inline)) {
                    constexpr int S = decltype(sc)::value;
                    if constexpr (S < NA) {
                        sb_step<MODE>(xr[S], yr[S], acc[S], c0, g, dt, dta0);
                        lds_store(wr[S] + XN, shared_value<MODE>(xr[S]));
                    }
                });
                __syncthreads();
            };
            // steps in runs between checkpoints; the buffer read at step k is k & 1
            int k = 0;
            while (k < B.K) {
                const int kend =
                    B.ckpt_every > 0 ? min(B.K, k - k % B.ckpt_every + B.ckpt_every) : B.K;
                if (k & 1) step(std::integral_constant<int, 1>{}, k++);
                for (; k + 1 < kend; k += 2) {
                    step(std::integral_constant<int, 0>{}, k);
                    step(std::integral_constant<int, 1>{}, k + 1);
                }
                if (k < kend) step(std::integral_constant<int, 0>{}, k++);
                if (B.ckpt_every > 0 && k % B.ckpt_every == 0) {
                    const double en = agent_energy(xs + (k & 1) * kStride);
                    const bool mine = t < A && agent0 + t < B.M;
                    if (mine)
                        B.etrace[(static_cast<size_t>(e) * B.n_ckpt + ck) * B.M + agent0 + t] = en;
                    stamp(ck + 1);
                    ++ck;
                    // target mode: the event's work stops at the first
                    // checkpoint where one of its agents (of this item or,
                    // through the event's flag, of another) reaches the target
                    if (B.target) {
                        // (an OR over the workgroup through the item word: the
                        // kernel keeps no static LDS, see the launch)
                        if (t == 0) *item_s = 0;
                        __syncthreads();
                        if (mine && en <= B.target[e]) *item_s = 1;
                        __syncthreads();
                        if (t == 0) {
                            const int hit = *item_s;
                            if (hit)
                                __hip_atomic_store(B.done + e, 1, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                            *item_s = hit || __hip_atomic_load(B.done + e, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                        }
                        __syncthreads();
                        const bool stop = *item_s != 0;
                        __syncthreads();
                        if (stop) break;
                    }
                }
            }
            k_done = k;
        };
        auto with_sh = [&](auto nac, auto c0c) __attribute__((always_inline)) {
            if (short_rest)
                run(nac, c0c, std::true_type{});
            else
                run(nac, c0c, std::false_type{});
        };
        auto with_c0 = [&](auto nac) __attribute__((always_inline)) {
            if (cap0 <= 4)
                with_sh(nac, std::integral_constant<int, 4>{});
            else if (cap0 <= 8)
                with_sh(nac, std::integral_constant<int, 8>{});
            else
                with_sh(nac, std::integral_constant<int, kCap[0]>{});
        };
        switch (n_act) {
            case 1: with_c0(std::integral_constant<int, 1>{}); break;
            case 2: with_c0(std::integral_constant<int, 2>{}); break;
            case 3: with_c0(std::integral_constant<int, 3>{}); break;
            case 4: with_c0(std::integral_constant<int, 4>{}); break;
            case 5: with_c0(std::integral_constant<int, 5>{}); break;
            case 6: with_c0(std::integral_constant<int, 6>{}); break;
            case 7: with_c0(std::integral_constant<int, 7>{}); break;
            case 8: with_c0(std::integral_constant<int, 8>{}); break;
            default: with_c0(std::integral_constant<int, kS>{}); break;
        }
        // checkpoints a target stop skipped read NaN (no state was reached)
        if (t < A && agent0 + t < B.M)
            for (int c = ck; c < B.n_ckpt; ++c) {
                B.etrace[(static_cast<size_t>(e) * B.n_ckpt + c) * B.M + agent0 + t] = NAN;
                if (B.ckpt_clock)
                    B.ckpt_clock[(static_cast<size_t>(e) * (B.n_ckpt + 1) + c + 1) * B.M + agent0 + t] = 0;
            }
        const float *xfin = xs + (k_done & 1) * kStride;
        const double en = agent_energy(xfin);
        if (t < A && agent0 + t < B.M) B.energy[static_cast<size_t>(e) * B.M + agent0 + t] = en;
        for_slots([&](auto sc) __attribute__((always_inline)) {
            constexpr int S = decltype(sc)::value;
            const int i = spin_of(S);
            if (i >= 0) {
                const size_t o = (static_cast<size_t>(E.row_off) + i) * B.M + agent;
                B.T[o] = xr[S] >= 0.0f ? 1 : 0;
                if (B.x_out) B.x_out[o] = xr[S];
            }
        });
        __syncthreads();
    }
}

// The step kernel of one mode, coupling format and workgroup shape (the
// launch's work counter must already be zero).
template <int MODE, int JP, int TPB>
hipError_t launch_batch_steps_tu(const BatchArgs &B, hipStream_t st) {
    const size_t lds = batch_lds_bytes(TPB, B.tail_cap);
    // the packed 16-bit neighbour addresses assume the dynamic LDS starts at
    // address 0, which holds when the kernel has no static LDS
    static const bool base_zero = [] {
        hipFuncAttributes fa{};
        return hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(sb_batch<MODE, JP, TPB>)) ==
                   hipSuccess &&
               fa.sharedSizeBytes == 0;
    }();
    if (!base_zero) return hipErrorInvalidConfiguration;
    return launch_with_lds(sb_batch<MODE, JP, TPB>, dim3(B.grid), dim3(TPB), lds, st, B);
}

}  // namespace sbt
