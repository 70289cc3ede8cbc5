// The whole batch (every stage of every view) in one persistent launch.
//
// Work items are chunks of up to `chunk` tiles of one view and one stage,
// handed out by one atomic counter in stage-major order (every view's SSAO
// prep, then every view's raw AO, ...).  A chunk of stage s of view v first
// waits until all chunks of the view's previous stage are done (per view and
// stage counters), so a view's shading can start while other views are still
// in SSAO, and no grid-wide barrier separates the stages.
//
// gfx950 notes:
//  * the L2 of each XCD is its own: finished chunks are published with an
//    agent-scope release fence (which writes the XCD's dirty L2 lines back)
//    before their counters are incremented, and a waiting block takes an
//    agent-scope acquire fence after it has seen the count, before any of its
//    threads reads the producer's data.  Both cost far more than a plain
//    atomic (about 20 ns per release over the whole device, measured), so a
//    block publishes its chunks in groups and, once it has seen a whole stage
//    (or one view's stage) complete, does not wait or fence again for it.
//  * deadlock freedom: chunks are handed out in stage-major order and a chunk
//    only waits for chunks handed out before it, which belong to running blocks
//    that never wait for later chunks; every wait is bounded (wait_limit polls),
//    and a block that gives up sets the error word, after which no block takes
//    new work, so the grid always drains.
//  * one block shape for every stage: 256 threads, the stage's tile function
//    as in the seven-launch form (SSAO raw and blur on 16 x 16 texel tiles,
//    composite on four 64 x 8 tiles, one per wavefront).  Per output value
//    the arithmetic is that of the other forms, so the results are bitwise equal.
#include "device_common.hpp"
#include "launch.hpp"
#include "post_tiles.hpp"
#include "shade_tiles.hpp"
#include "ssao_tiles.hpp"

namespace epb {

union PersistLds {
    struct {
        float sd[blur_lds_rows<kPersistSsaoT, kPersistSsaoT>()][kPersistSsaoT + 3];
        float sa[blur_lds_rows<kPersistSsaoT, kPersistSsaoT>()][kPersistSsaoT + 3];
    } blur;
    DownLds down;
    BlurLds bloom;
};

__device__ __forceinline__ int *persist_done(PersistState *st) { return reinterpret_cast<int *>(st + 1); }

// The previous stage of view v that has work, or -1.
__device__ __forceinline__ int prev_stage(const void *table, int v, int s) {
    for (int p = s - 1; p >= 0; --p) {
        const int *cs = batch_cstart(table, p);
        if (cs[v + 1] > cs[v]) return p;
    }
    return -1;
}

// One tile of stage s of view d (uniform across the block).  T is the storage
// type of the G-buffer, AO and HDR; TP that of the bloom pyramid texels.
template <typename T, typename TP>
__device__ __forceinline__ void persist_tile(const BatchHeader *h, const ViewDesc &d, int s, int t, PersistLds &sm) {
    switch (s) {
    case kStPrep: ssao_prep_item(d.ssao, t); break;
    case kStRaw:  // raw AO goes to float scratch when a blur follows
        if (h->blur) ssao_raw_tile<kPersistSsaoT, kPersistSsaoT, 8, T, float>(d.ssao, t);
        else ssao_raw_tile<kPersistSsaoT, kPersistSsaoT, 8, T, T>(d.ssao, t);
        break;
    case kStBlur: ssao_blur_tile<kPersistSsaoT, kPersistSsaoT, T>(d.ssao, t, sm.blur.sd, sm.blur.sa); break;
    case kStShade: shade_tile<32, 8, false, T, T, T>(d.shade, t); break;
    case kStDown: bloom_down_tile<T, TP>(d.post, t, sm.down); break;
    case kStBloomBlur: bloom_blur_item<TP>(d.post, t, sm.bloom); break;
    default: {
        int tiles = ((d.post.W + kPostTx - 1) / kPostTx) * ((d.post.H + kPostTy - 1) / kPostTy);
        int tile = t * kPersistCompositeTiles + (int)(threadIdx.x / kPostTx);
        if (tile < tiles) composite_tile<T, TP>(d.post, tile, (int)(threadIdx.x % kPostTx));
    }
    }
}

__global__ void __launch_bounds__(256) k_persist_clear(int *state, int n) {
    for (int i = (int)threadIdx.x; i < n; i += 256) state[i] = 0;
}

// Finished chunks a block has not published yet (thread 0 only): one stage,
// up to kPending views.
constexpr int kPending = 32;
struct Pending {
    int v[kPending], n[kPending];
};

// Publishes the pending chunks: one release fence (the expensive part), then
// the per-view and per-stage counts.
__device__ __forceinline__ void publish(PersistState *st, int *done, Pending &pd, int &np, int stage) {
    if (np == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    int total = 0;
    for (int i = 0; i < np; ++i) {
        __hip_atomic_fetch_add(&done[pd.v[i] * kStages + stage], pd.n[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        total += pd.n[i];
    }
    __hip_atomic_fetch_add(&st->stage_done[stage], total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    np = 0;
}

// Every stage's code in one kernel: it needs at least the largest register
// count of any stage (the composite's 91-96), and the combined kernel spills
// heavily at 5 waves per SIMD (96 registers), so it runs at 4 waves per SIMD
// with 128 registers (a few registers still spill).
//
// A block publishes its finished chunks lazily: when it moves to another stage,
// before it waits for anything, when its pending list is full and when it
// exits.  Consumers of a stage's chunks are handed out only after every chunk
// of that stage, so the delay is at most the block's current chunk, while the
// release fences drop from one per chunk to about one per block and stage.  A
// block never waits with unpublished work, so the order argument above holds.
template <typename T, typename TP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_batch_persistent(const void *__restrict__ table, PersistState *__restrict__ st) {
    __shared__ PersistLds sm;
    __shared__ Pending pd;
    __shared__ int s_chunk, s_go;
    const BatchHeader *h = (const BatchHeader *)table;
    const ViewDesc *views = batch_views(table);
    int *done = persist_done(st);
    const int n = h->n_views;
    // thread 0: dependencies this block has already seen complete (after an acquire),
    // and its unpublished chunks (all of stage pend_s)
    unsigned stage_complete = 0;
    int seen_v = -1, seen_s = -1, np = 0, pend_s = -1;
    for (;;) {
        if (threadIdx.x == 0) {
            int g = __hip_atomic_fetch_add(&st->head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_load(&st->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) g = h->total_chunks;
            if (g >= h->total_chunks) publish(st, done, pd, np, pend_s);
            s_chunk = g;
        }
        __syncthreads();
        const int g = s_chunk;
        if (g >= h->total_chunks) break;
        int s = 0;
        while (g >= h->chunk_first[s + 1]) ++s;
        const int *cs = batch_cstart(table, s);
        const int local = g - h->chunk_first[s];
        const int v = find_view(cs, n, local);
        const int c = local - cs[v];
        if (threadIdx.x == 0) {
            if (s != pend_s) publish(st, done, pd, np, pend_s);
            int ok = 1;
            int p = prev_stage(table, v, s);
            if (p >= 0 && !((stage_complete >> p) & 1u) && !(seen_v == v && seen_s == p)) {
                publish(st, done, pd, np, pend_s);
                const int *cp = batch_cstart(table, p);
                const int need = cp[v + 1] - cp[v];
                const int stage_need = h->chunk_first[p + 1] - h->chunk_first[p];
                ok = 0;
                for (int k = 0; k < h->wait_limit; ++k) {
                    if (h->gate) {
                        if (__hip_atomic_load(&st->stage_done[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                            stage_need) {
                            stage_complete |= 1u << p;
                            ok = 1;
                            break;
                        }
                        if (__hip_atomic_load(&done[v * kStages + p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                            need) {
                            seen_v = v;
                            seen_s = p;
                            ok = 1;
                            break;
                        }
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
                if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                else __hip_atomic_store(&st->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            s_go = ok;
        }
        __syncthreads();
        if (!s_go) break;
        const int *sv = batch_start(table, s);
        const int items = sv[v + 1] - sv[v];
        const int t0 = c * h->chunk, t1 = min(t0 + h->chunk, items);
        for (int t = t0; t < t1; ++t) persist_tile<T, TP>(h, views[v], s, t, sm);
        __syncthreads();  // every thread's stores of the chunk precede its publication
        if (threadIdx.x == 0) {
            if (np > 0 && pd.v[np - 1] == v) {
                ++pd.n[np - 1];
            } else {
                if (np == kPending) publish(st, done, pd, np, pend_s);
                pd.v[np] = v;
                pd.n[np] = 1;
                ++np;
            }
            pend_s = s;
        }
    }
}

// Workgroups of the persistent grid: blocks_per_cu per CU, or as many as fit.
template <typename T, typename TP>
static hipError_t persist_grid(const BatchHeader &h, int *grid) {
    int dev = 0, cus = 0, per_cu = h.blocks_per_cu;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && per_cu <= 0)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent<T, TP>, 256, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    *grid = per_cu * (cus > 0 ? cus : 256);
    if (*grid > h.total_chunks) *grid = h.total_chunks > 0 ? h.total_chunks : 1;
    return hipSuccess;
}

template <typename T, typename TP>
static hipError_t go_persistent(const BatchHeader &h, const void *table, hipStream_t s) {
    int grid = 0;
    hipError_t e = persist_grid<T, TP>(h, &grid);
    if (e != hipSuccess) return e;
    PersistState *st = (PersistState *)((char *)const_cast<void *>(table) + batch_state_offset(h.n_views));
    int words = (int)((sizeof(PersistState) + sizeof(int) * kStages * (size_t)h.n_views) / sizeof(int));
    hipLaunchKernelGGL(k_persist_clear, dim3(1), dim3(256), 0, s, (int *)st, words);
    hipLaunchKernelGGL((k_batch_persistent<T, TP>), dim3(grid), dim3(256), 0, s, table, st);
    return hipGetLastError();
}

hipError_t launch_persistent(const BatchHeader &h, const void *table, hipStream_t s) {
    return h.gdtype == EPB_F32 ? go_persistent<float, float4>(h, table, s) : go_persistent<__half, Half4>(h, table, s);
}

}  // namespace epb
