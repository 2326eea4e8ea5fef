// batch.hpp -- batched evaluation of many independent problems of uneven sizes.
//
// The work of a batch is a list of tasks: a task is a run of consecutive tiles
// (blocks of the single-problem launches) of one pass of one problem, grouped so
// that one 256-thread block carries several small tiles at once.  Task lists are
// pass-major (all P1 tasks, then all P2 tasks, ...), so every task depends only
// on tasks before it.
//
//   queue schedule : ONE persistent launch.  Each die (XCD) serves a task queue of
//                    the problems pinned to it; before a task of pass p a block
//                    waits until every task of the preceding pass of the same
//                    problem is done (per-problem counters).  A block only waits on
//                    tasks claimed earlier by running blocks of its die, so the
//                    launch cannot deadlock whatever the number of resident blocks.
//                    The last block to leave clears the counters for the next launch.
//   phased schedule: one launch per pass type over the tasks of that pass; kernel
//                    boundaries carry the dependencies (also per pass and size).
//
// The tile code is the single-problem code, so every problem's result is bitwise
// that of its own evaluation, under any schedule.
#pragma once

#include <hip/hip_runtime.h>

#include "passes.hpp"

namespace gsk {

constexpr int BATCH_THREADS = 256;

struct BatchProblem {
    int n, d, mode;            // mode: SPEC_PLAIN / SPEC_DIPOLAR
    const double* rho;
    double* u;
    cpx* X1;
    cpx* X2;
    const double* spec;
    const cpx* tw;
    DipoleArgs dip;
};

struct BatchTask {
    int prob, pass;            // problem index, pass 1..5
    int tile0, tile1;          // tiles tile0 .. tile1 - 1 of that pass
    int dep_pass, dep_count;   // wait until dep_count tasks of pass dep_pass of this problem are done (0: none)
};

// Task queues of the queue schedule: one per XCD (accelerator die) in use.  qmap maps
// a hardware XCC id (0..15) to its queue (-1: none); queue q holds tasks
// qoff[q] .. qoff[q+1]-1.  local: every problem's tasks sit in one queue, so a
// producer and its consumers share one L2 and the dependencies need no L2
// write-back; otherwise (one queue for all dies) agent-scope release/acquire.
constexpr int BATCH_MAX_QUEUES = 16;
struct BatchQueues {
    int nq, local;
    int qmap[BATCH_MAX_QUEUES];
    int qoff[BATCH_MAX_QUEUES + 1];
};

// Counters of the queue schedule: [0] blocks that left, [1 + q] next task of queue q,
// [1 + BATCH_MAX_QUEUES + 8 b + p] tasks of pass p of problem b that are done; one
// more word after them is the error flag (a dependency wait gave up, or a queue was
// left unfinished because no block ran on its die), which launches do not clear.
__host__ __device__ constexpr int batch_counter(int prob, int pass) { return 1 + BATCH_MAX_QUEUES + 8 * prob + pass; }

// Hardware id of the XCD the calling wave runs on (HW_REG_XCC_ID, bits 3:0).
__device__ __forceinline__ int hw_xcc_id() { return (int)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20); }

// Threads and LDS slots of one tile of pass p at size N; tiles per problem.
// P5 tiles take the single-problem kernel's split form where it has one (the two halves of
// the padded inverse on the two lane halves of every wave: twice the threads and LDS areas
// per tile, the same LDS per block, E complex values fewer live per thread).
template <int N> __host__ __device__ constexpr int tile_threads(int pass) {
    return pass == 1 ? Geo<N>::TX
                     : (pass == 5 ? p5_threads<N, Geo<N>::PPX>() : (pass == 3 ? Geo<N>::TZ : Geo<N>::TY));
}
template <int N> __host__ __device__ constexpr int tile_lds(int pass) {
    return pass == 3   ? 2 * Geo<N>::PPZ * Geo<N>::AZ
           : pass == 1 ? Geo<N>::PPX * Geo<N>::A
           : pass == 5 ? (p5_split<N, Geo<N>::PPX>() ? 2 : 1) * Geo<N>::PPX * Geo<N>::A
                       : Geo<N>::PPY * Geo<N>::A;
}
template <int N> __host__ __device__ inline int tile_count(int pass, int d) {
    using Gm = Geo<N>;
    if (pass == 1 || pass == 5) return ((N + 2 * Gm::PPX - 1) / (2 * Gm::PPX)) * (d == 3 ? N : 1);
    if (pass == 2 || pass == 4) return ((N + Gm::PPY - 1) / Gm::PPY) * (N + 1);
    const int np = (d == 3) ? (N + 1) * 2 * N : N + 1;
    return (np + Gm::PPZ - 1) / Gm::PPZ;
}

// sizes a batch may hold
#define GS_BATCH_SIZES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

template <int N> constexpr int batch_lds_of() {
    int m = 0;
    for (int p = 1; p <= 5; ++p) {
        const int s = tile_lds<N>(p) * (BATCH_THREADS / tile_threads<N>(p));
        m = s > m ? s : m;
    }
    return m;
}
#define GS_LDS_OF(N) batch_lds_of<N>(),
constexpr int batch_lds_slots() {
    constexpr int v[] = {GS_BATCH_SIZES(GS_LDS_OF) 0};
    int m = 0;
    for (int x : v) m = x > m ? x : m;
    return m;
}
#undef GS_LDS_OF

// Tiles tile0 .. tile0 + (block / tile threads) - 1 of pass PASS of one problem.
template <int N, int PASS>
__device__ __forceinline__ void batch_tile(const BatchProblem& P, int tile0, int tile1, cpx* lds) {
    constexpr int T = tile_threads<N>(PASS);
    static_assert(BATCH_THREADS % T == 0, "tile threads must divide the block");
    // the thread index is laundered so that nothing derived from it is hoisted out
    // of the task loop (kept live across every size and pass, that would spill)
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    const int sub = lane / T, tid = lane % T;
    const int tile = tile0 + sub;
    const bool active = tile < tile1;
    cpx* l = lds + sub * tile_lds<N>(PASS);
    using Gm = Geo<N>;
    // descriptor pointers typed as global memory (global, not flat, accesses)
    const gp<const double> rho = (gp<const double>)P.rho;
    const gp<double> u = (gp<double>)P.u;
    const gp<cpx> X1 = (gp<cpx>)P.X1;
    const gp<cpx> X2 = (gp<cpx>)P.X2;
    const gp<const double> spec = (gp<const double>)P.spec;
    const gp<const cpx> tw = (gp<const cpx>)P.tw;
    if constexpr (PASS == 1 || PASS == 5) {
        constexpr int nbx = (N + 2 * Gm::PPX - 1) / (2 * Gm::PPX);
        const int bx = tile % nbx, z = tile / nbx;
        if constexpr (PASS == 1) x_r2c_tile<N, NT_P1, true, Gm::PPX, true>(rho, X1, tw, bx, z, tid, active, l);
        else if constexpr (p5_split<N, Gm::PPX>())
            x_c2r_tile_split<N, NT_P5, false, Gm::PPX>(X1, u, tw, bx, z, tid, l, 1.0, active);
        else x_c2r_tile<N>(X1, u, tw, bx, z, tid, active, l);
    } else if constexpr (PASS == 2 || PASS == 4) {
        constexpr int nbz = (N + Gm::PPY - 1) / Gm::PPY;
        const int bx = tile % nbz, kxl = tile / nbz;
        if constexpr (PASS == 2) y_fwd_tile<N>(X1, X2, tw, 0, bx, kxl, tid, active, l);
        else y_inv_tile<N>(X2, X1, tw, 0, bx, kxl, tid, active, l);
    } else {
        if (P.d == 3) {
            const int np = (N + 1) * 2 * N;
            if (P.mode == SPEC_DIPOLAR)
                fused_group<N, 3, SPEC_DIPOLAR>(X2, spec, tw, np, 0, P.dip, tile, tid, active, l);
            else
                fused_group<N, 3, SPEC_PLAIN>(X2, spec, tw, np, 0, P.dip, tile, tid, active, l);
        } else {
            fused_group<N, 2, SPEC_PLAIN>(X1, spec, tw, N + 1, 0, P.dip, tile, tid, active, l);
        }
    }
}

// All tiles of one task, one block-full at a time.
template <int N, int PASS>
__device__ __forceinline__ void batch_run(const BatchProblem& P, int tile0, int tile1, cpx* lds) {
    constexpr int sub = BATCH_THREADS / tile_threads<N>(PASS);
    for (int j = tile0; j < tile1; j += sub) {
        batch_tile<N, PASS>(P, j, tile1, lds);
        lds_barrier();      // the next tiles reuse the LDS
    }
}

template <int PASS>
__device__ __forceinline__ void batch_task_pass(const BatchProblem& P, const BatchTask& t, cpx* lds) {
    switch (P.n) {
#define GS_CASE(N) \
    case N: batch_run<N, PASS>(P, t.tile0, t.tile1, lds); break;
        GS_BATCH_SIZES(GS_CASE)
#undef GS_CASE
        default: break;
    }
}

__device__ __forceinline__ void batch_task(const BatchProblem& P, const BatchTask& t, cpx* lds) {
    switch (t.pass) {
        case 1: batch_task_pass<1>(P, t, lds); break;
        case 2: batch_task_pass<2>(P, t, lds); break;
        case 3: batch_task_pass<3>(P, t, lds); break;
        case 4: batch_task_pass<4>(P, t, lds); break;
        case 5: batch_task_pass<5>(P, t, lds); break;
        default: break;
    }
}

// The union kernels (every size's tile code in one function) are held to three waves per
// SIMD, which their LDS (three blocks per CU) allows: 168 VGPRs with a few dozen bytes of
// spill in the 96-point dipolar fused code, against 225 VGPRs (two waves) unbounded; the tile
// codes keep fewer values live for this (P1 loads its rows again for the second half, P5
// runs the split form).  Measured on the 64-problem workload: queue 2.66 -> 2.52 ms, phased
// 2.52 -> 2.41 ms, the same bits.
constexpr int BATCH_UNION_WAVES = 3;

// Phased schedule: the tasks of one pass, block-strided.
template <int PASS>
__global__ void __launch_bounds__(BATCH_THREADS) __attribute__((amdgpu_waves_per_eu(BATCH_UNION_WAVES))) k_batch_pass(const BatchProblem* __restrict__ probs,
                                                              const BatchTask* __restrict__ tasks, int ntasks) {
    __shared__ cpx lds[batch_lds_slots()];
    for (int k = blockIdx.x; k < ntasks; k += gridDim.x) {
        const BatchTask t = tasks[k];
        batch_task_pass<PASS>(probs[t.prob], t, lds);
    }
}

// Phased-by-size schedule: one launch per pass and per grid size over that size's
// tasks (each launch gets the register allocation of its own tile code).
template <int N, int PASS>
__global__ void __launch_bounds__(BATCH_THREADS) k_batch_size(const BatchProblem* __restrict__ probs,
                                                              const BatchTask* __restrict__ tasks, int ntasks) {
    __shared__ cpx lds[batch_lds_of<N>()];
    for (int k = blockIdx.x; k < ntasks; k += gridDim.x) {
        const BatchTask t = tasks[k];
        batch_run<N, PASS>(probs[t.prob], t.tile0, t.tile1, lds);
    }
}

// Queue schedule: one persistent launch over every task of the batch.
//
// A block serves the queue of the die it runs on.  Every branch of the task loop is
// wave-uniform (conditions pass through readfirstlane): wave 0 of the block does the
// counter work with all its lanes, lane 0 contributing the increment and the others
// zero.  A lane-0-only branch at the loop boundary would let the compiler park lane
// 0 outside the loop while the other lanes of its wave run on through the barriers
// with a stale task index.
//
// Memory ordering, local queues: the producer's stores reach the die's L2 before
// its counter increment (every wave waits for its stores before the block barrier;
// the vector L1 is write through), and a consumer invalidates its own L1 after
// observing the counter.
// Otherwise agent-scope release (L2 write-back) and acquire (L2 invalidate).
//
// A dependency wait gives up after spin_limit polls (far beyond any task's
// duration): it raises the error flag ctr[nctr] and carries on, so every wave
// reaches the end of the launch whatever happens; the host reads the flag.
__global__ void __launch_bounds__(BATCH_THREADS) __attribute__((amdgpu_waves_per_eu(BATCH_UNION_WAVES))) k_batch_queue(const BatchProblem* __restrict__ probs,
                                                               const BatchTask* __restrict__ tasks, BatchQueues Q,
                                                               unsigned* __restrict__ ctr, int nctr,
                                                               unsigned spin_limit) {
    __shared__ cpx lds[batch_lds_slots()];
    __shared__ int s_task, s_next;
    const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) < 64u;
    const unsigned one = (threadIdx.x == 0) ? 1u : 0u;      // the increment of lane 0
    const int q = Q.nq == 1 && !Q.local ? 0 : Q.qmap[hw_xcc_id() & (BATCH_MAX_QUEUES - 1)];
    const int base = q >= 0 ? Q.qoff[q] : 0;
    const int count = q >= 0 ? Q.qoff[q + 1] - base : 0;
    unsigned* head = &ctr[1 + (q >= 0 ? q : 0)];
    if (wave0) {
        int k0 = count;
        if (count > 0)
            k0 = (int)__builtin_amdgcn_readfirstlane(
                __hip_atomic_fetch_add(head, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        s_task = k0;
    }
    __syncthreads();
    for (;;) {
        const int k = __builtin_amdgcn_readfirstlane(s_task);
        if (k >= count) break;
        const BatchTask t = tasks[base + k];
        if (wave0) {
            // claim the next task now: its index arrives while this one waits and runs
            // (a claimed task depends only on tasks before it in its queue, so claiming
            // early cannot deadlock)
            const unsigned nx = __hip_atomic_fetch_add(head, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t.dep_count > 0) {
                unsigned* c = &ctr[batch_counter(t.prob, t.dep_pass)];
                for (unsigned polls = 0;; ++polls) {
                    const unsigned done =
                        __builtin_amdgcn_readfirstlane(__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (done >= (unsigned)t.dep_count) break;
                    if (polls >= spin_limit) {
                        __hip_atomic_store(&ctr[nctr], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (Q.local) asm volatile("buffer_inv sc0" ::: "memory");        // this CU's L1
                else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_next = (int)__builtin_amdgcn_readfirstlane(nx);
        }
        __syncthreads();
        batch_task(probs[t.prob], t, lds);
        // every wave waits until its stores are complete (in the die's L2; the block
        // barrier alone orders LDS only), then the barrier
        __builtin_amdgcn_s_waitcnt(0x0F70);    // vmcnt(0)
        __syncthreads();
        if (wave0) {
            unsigned* c = &ctr[batch_counter(t.prob, t.pass)];
            if (Q.local) __hip_atomic_fetch_add(c, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else __hip_atomic_fetch_add(c, one, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            s_task = s_next;
        }
        __syncthreads();
    }
    // the last block to leave checks that every queue was drained and clears the
    // counters (the next launch starts after this one ends)
    if (wave0) {
        const unsigned e = __hip_atomic_fetch_add(&ctr[0], one, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_task = (__builtin_amdgcn_readfirstlane(e) == gridDim.x - 1u) ? 1 : 0;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_task)) {
        if (wave0) {
            bool drained = true;
            for (int i = 0; i < Q.nq; ++i)
                drained = drained && __hip_atomic_load(&ctr[1 + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                                         (unsigned)(Q.qoff[i + 1] - Q.qoff[i]);
            if (!__builtin_amdgcn_readfirstlane(drained ? 1u : 0u))
                __hip_atomic_store(&ctr[nctr], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int i = threadIdx.x; i < nctr; i += BATCH_THREADS)
            __hip_atomic_store(&ctr[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace gsk
