// common.h -- internal declarations shared by the gfx950 kernels and the C-ABI host code.
//
// Layout decisions (all FP64 unless stated):
//   - Problems are stored back to back; work is cut into tiles of 64 consecutive entries
//     (roots or poles) of one problem, one wavefront lane per entry.
//   - Kernels read the per-pole data of a problem with wave-uniform indices, so the
//     compiler serves them from the scalar data cache and every lane reuses them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/superdc.h"

namespace sdc {

constexpr int WAVE = 64;       // CDNA wavefront width
constexpr int TILE = 64;       // entries per work tile
constexpr int SEC_CHUNK = 512; // roots per work item of the secular solver

struct Tile {
    int32_t prob;  // problem index
    int32_t row0;  // first local row of the tile
};

// self-resetting work queue of a persistent launch (two counters, zero between launches)
struct Queue {
    unsigned int next;
    unsigned int done;
};

// ----------------------------------------------------------------------------------
// device helpers
// ----------------------------------------------------------------------------------

// 1/t from the hardware reciprocal estimate refined by two Newton steps
// r <- r + r (1 - t r); each step squares the relative error.
__device__ __forceinline__ double rcp_nr(double t) {
    double r = __builtin_amdgcn_rcp(t);
    double e = __builtin_fma(-t, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-t, r, 1.0);
    r = __builtin_fma(r, e, r);
    return r;
}

// clamp a caller-supplied local index into [0, n) so a bad origin array cannot read
// outside its problem
__device__ __forceinline__ int clamp_idx(int K, int n) { return K < 0 ? 0 : (K >= n ? n - 1 : K); }

// the same with a single Newton step (relative error <= ~11 ulp on gfx950)
__device__ __forceinline__ double rcp_nr1(double t) {
    const double r = __builtin_amdgcn_rcp(t);
    return __builtin_fma(r, __builtin_fma(-t, r, 1.0), r);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// Let the last v_mfma_f64_16x16x4f64 of a chain finish before its accumulators are read
// by other instructions: on gfx950 it occupies the matrix pipe for 64 cycles, longer than
// the wait states the compiler puts between it and such a read, which shows as stale
// accumulators when the SIMD has no other wavefront to issue meanwhile.  ~128 cycles.
__device__ __forceinline__ void mfma_drain() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_sleep(2);
    __builtin_amdgcn_sched_barrier(0);
}

// This wavefront's instruction-issue priority among the SIMD's wavefronts (0 lowest, 3
// highest); p must be wave-uniform.
__device__ __forceinline__ void wave_priority(int p) {
    if (p <= 0) __builtin_amdgcn_s_setprio(0);
    else if (p == 1) __builtin_amdgcn_s_setprio(1);
    else if (p == 2) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(3);
}

template <typename T>
__device__ __forceinline__ T wave_uniform(T v) {
    return __builtin_amdgcn_readfirstlane(v);
}

// Read-only data indexed by a wave-uniform index: going through the constant address
// space lets the compiler fetch it with scalar loads into SGPRs (one fetch feeds all 64
// lanes, and the vector memory path stays free).  Only for data no kernel of the same
// launch writes.
typedef const __attribute__((address_space(4))) double *const_double_ptr;

__device__ __forceinline__ const_double_ptr as_const(const double *p) {
    return (const_double_ptr)p;
}
// packed pairs / quads read component-wise (adjacent scalar loads merge into one fetch)
struct cpair {
    const_double_ptr p;
    __device__ __forceinline__ double2 operator[](int j) const {
        return make_double2(p[2 * j], p[2 * j + 1]);
    }
};
struct cquad {
    const_double_ptr p;
    __device__ __forceinline__ double4 operator[](int j) const {
        return make_double4(p[4 * j], p[4 * j + 1], p[4 * j + 2], p[4 * j + 3]);
    }
};
__device__ __forceinline__ cpair as_const(const double2 *p) { return cpair{(const_double_ptr)p}; }
__device__ __forceinline__ cquad as_const(const double4 *p) { return cquad{(const_double_ptr)p}; }
typedef cpair const_double2_ptr;
typedef cquad const_double4_ptr;

// Orders one wavefront's LDS accesses across this point, for lanes that exchange data through
// LDS without the rest of the workgroup (a wavefront's LDS operations complete in program
// order; the fences keep the compiler from moving accesses across)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pull the next work item from a persistent queue (called by whole wavefront-0 of a WG
// and broadcast through LDS).  Returns -1 when the queue is drained.
__device__ __forceinline__ int queue_pull(Queue *q, int nitems, int *slot) {
    if (threadIdx.x == 0) *slot = (int)atomicAdd(&q->next, 1u);
    __syncthreads();
    int it = __builtin_amdgcn_readfirstlane(*slot);
    __syncthreads();
    return it < nitems ? it : -1;
}

// The last workgroup to leave resets the counters, so the next launch (or graph replay)
// starts from zero without a memset.
__device__ __forceinline__ void queue_leave(Queue *q) {
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned prev = atomicAdd(&q->done, 1u);
        if (prev == gridDim.x - 1) {
            atomicExch(&q->next, 0u);
            atomicExch(&q->done, 0u);
            __threadfence();
        }
    }
}

// The work items of a launch with one call site of the body: persistent (q != nullptr)
// workgroups pull items until the queue runs dry and then leave it; otherwise workgroup b
// takes item b.  One inlined copy of a large body (rather than one per branch) keeps a
// kernel's code within the instruction cache.
template <class Body>
__device__ __forceinline__ void for_each_item(Queue *q, int nitems, int *slot, Body &&body) {
    int item = q ? queue_pull(q, nitems, slot) : ((int)blockIdx.x < nitems ? (int)blockIdx.x : -1);
    while (item >= 0) {
        body(item);
        item = q ? queue_pull(q, nitems, slot) : -1;
    }
    if (q) queue_leave(q);
}

// ----------------------------------------------------------------------------------
// optional per-kernel timing (trace.cpp): a scope records HIP events around one launch
// ----------------------------------------------------------------------------------
enum KernelId : int {
    KID_VALIDATE = 0, KID_FMM_BOXES, KID_FMM_LISTS, KID_SECULAR, KID_SECULAR_FMM, KID_PACK,
    KID_LOEWNER, KID_BNORM, KID_APPLY_MFMA, KID_APPLY_VALU, KID_BWD, KID_BWD_RHO, KID_LEAF,
    KID_MERGE, KID_ASSEMBLE, KID_PERMUTE, KID_LEAF_APPLY, KID_STATUS_OR, KID_FILL,
    KID_LEAF_VECTORS, KID_FMMV_PACK, KID_FMMV_SOURCES, KID_FMMV_EVAL,
    KID_FMMV_EVAL_MFMA, KID_FMML_PACK, KID_FMML_MOMENTS, KID_LOEWNER_FMM, KID_DEFLATE,
    KID_DEFL_PLACE, KID_DEFL_ROTATE, KID_COPY_ROWS, KID_FMM_LOCAL, KID_DIVIDE, KID_SORT, KID_COUNT
};

// device counters of kernel `kid` while kernel timing is on (the current device), else
// nullptr: TRACE_WORDS words, [0] its work (pair evaluations or flops), and for the solvers
// [1] the live lanes summed over every pass of every wavefront, [2] the lanes those
// passes had (64 per wavefront pass)
constexpr int TRACE_WORDS = 4;
unsigned long long *trace_work(int kid);

class TraceScope {
  public:
    TraceScope(int kid, hipStream_t s);
    ~TraceScope();

  private:
    int kid_;
    hipStream_t s_;
    hipEvent_t e0_ = nullptr, e1_ = nullptr;
};

// a kernel launch bracketed by the trace scope of kernel id KID
#define SDC_LAUNCH(KID, KERNEL, GRID, BLOCK, LDS, STREAM, ...)                     \
    do {                                                                          \
        ::sdc::TraceScope trace_scope_(KID, STREAM);                              \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, __VA_ARGS__);        \
    } while (0)

}  // namespace sdc

// ----------------------------------------------------------------------------------
// host-side objects
// ----------------------------------------------------------------------------------
#ifdef __cplusplus
#include <vector>

enum WsSlot {
    WS_DW = 0, WS_KE = 1, WS_DZ = 2, WS_Z2 = 3, WS_BK = 4, WS_BP = 5, WS_TMP = 6, WS_VPAIR = 7,
    WS_VSRC = 8, WS_DEFL_VAL = 9, WS_DEFL_FLAG = 10, WS_DEFL_T = 11, WS_DEFL_SEGI = 12,
    WS_DEFL_SEGD = 13, kNumWs
};

struct superdc_ctx {
    int device = 0;
    int num_cu = 256;
    // grow-only workspace buffers
    void *ws[kNumWs] = {nullptr};
    size_t ws_cap[kNumWs] = {0};
    sdc::Queue *queues = nullptr;  // kNumQueues counters, zeroed at creation
    int fmm_crossover = 1024;      // automatic method: FMM for problems at least this large (measured)
};

enum QueueSlot {
    Q_SECULAR = 0, Q_LOEWNER, Q_BNORM, Q_APPLY, Q_BWD1, Q_BWD2, Q_VALIDATE, Q_SECULAR_FMM,
    Q_FMMV, kNumQueues
};

namespace sdc {
struct FmmPlan;
}

// Work items of one cut length: longest problems first (persistent launches) and in
// problem order (plain launches; problem p owns nat[begin[p] .. begin[p+1])).
struct TileList {
    sdc::Tile *lpt = nullptr;
    sdc::Tile *nat = nullptr;
    int32_t count = 0;
    std::vector<int32_t> begin;
};

// launch shape of one kernel family: entries per work item and wavefronts per item
struct LaunchShape {
    int chunk = 0;
    int split = 1;
};

struct superdc_batch {
    superdc_ctx *ctx = nullptr;
    int32_t nprob = 0;
    int64_t total = 0;
    int32_t max_n = 0;
    std::vector<int64_t> off_h;
    int64_t *off_d = nullptr;
    std::vector<int> order;             // problems, longest first
    TileList lists[4];                  // cut lengths 64, 128, 256, 512
    // chosen launch shapes (heuristic, or set by the autotuner): persistent launches
    LaunchShape sec, vec, app, bwd;
    int fmm_ssplit = 0;                 // FMM solver: wavefronts per work item (0: heuristic)
    bool tuned = false;
    // triangular-FMM layout (built on the first FMM solve; see fmm.h)
    sdc::FmmPlan *fmm = nullptr;
    // validation of long problems: slices per problem and their partial sums
    int vsplit = 1;
    double *vsum = nullptr;     // [nprob][vsplit]
    int32_t *vst = nullptr;     // [nprob][vsplit]
};

namespace sdc {
// the tile list of a given cut length (64, 128, 256 or 512), built on first use
const TileList *tile_list(superdc_batch *b, int chunk);
// SUPERDC_OK or SUPERDC_EINVAL for an options struct
int opts_check(const superdc_opts *o);
// grid of a persistent launch: per_cu workgroups per CU, at most one per work item
int persistent_grid(const superdc_ctx *ctx, int ntiles, int per_cu);
// problems of at least this many roots use the triangular FMM under these options
int fmm_crossover_of(const superdc_ctx *ctx, const superdc_opts &o);
// launch shape of the plain (one launch per problem) direct solve of an n-root problem
::LaunchShape plain_shape(const superdc_ctx *ctx, int64_t n);
// the allocation-free solve's scratch array: its address on `device` is looked up once
// (noalloc.hip); called by superdc_create with that device current
int noalloc_init(int device);
}  // namespace sdc

namespace sdc {
// Loewner/b and the Cauchy apply behind superdc_loewner / superdc_cauchy_apply.
// reuse_lists: the batch's FMM interaction lists were built by a solve on the same poles
// d (internal callers that know it).  fmm_b = false leaves b to the next apply_run with
// fuse_b = true (Qhat^T X, 1 <= m < 16 columns, on the MFMA kernels), whose products form
// b beside the columns (from the same equivalent sources for the FMM problems) and write
// it to bnorm.
int loewner_run(superdc_ctx *ctx, const superdc_batch *b, const double *d, const double *z,
                const double *rho, const double *eta, const int32_t *origin,
                const int32_t *status, double *zhat, double *bnorm, const superdc_opts *opts,
                void *stream, bool reuse_lists, bool fmm_b = true);
int apply_run(superdc_ctx *ctx, const superdc_batch *b, const double *d, const double *zhat,
              const double *bnorm, const double *eta, const int32_t *origin,
              const int32_t *status, int trans, int32_t m, const double *X, int64_t ldx,
              double *Y, int64_t ldy, const superdc_opts *opts, void *stream, bool reuse_lists,
              bool fuse_b = false);

// grow a workspace slot to at least `bytes`; returns nullptr on allocation failure
void *ws_get(superdc_ctx *ctx, int slot, size_t bytes);

// kernel launchers (implemented next to their kernels); return hipError_t
struct SolveArgs {
    const int64_t *off;
    const Tile *tiles;
    int ntiles;
    const double *d, *z, *rho;
    double2 *dw;     // workspace (d_j, w_j)
    double *z2;      // workspace sum_j w_j per problem
    double2 *ke;     // workspace (d_{K_k}, eta_k) per root
    double *lam, *eta;
    int32_t *origin, *iters, *status;
    double stop_c;
    int max_iter;
    int chunk;       // roots per work item (the tile list is cut at this length)
    unsigned long long *work;  // when kernel timing is on: pole-root pair evaluations
    int unshifted;   // ablation: iterate on lambda itself, every difference d_j - lambda
    int hybrid;      // interpolation: 0 middle way, 1 the middle-way / fixed-weight hybrid
};
// validation and packing of problems [prob_first, prob_first + nprob); with vsplit > 1 each
// problem is cut into vsplit slices, one workgroup each, whose partial sums go to vsum/vst
// ([nprob][vsplit], indexed by problem) and are added in slice order by a second launch
hipError_t launch_validate(const SolveArgs &a, int prob_first, int nprob, int max_n, hipStream_t s,
                           int vsplit = 1, double *vsum = nullptr, int32_t *vst = nullptr);
hipError_t launch_secular(const SolveArgs &a, int split, Queue *q, int grid, hipStream_t s);

struct VecArgs {
    const int64_t *off;
    const Tile *tiles;
    int ntiles;
    const double *d, *z, *rho, *eta;
    const int32_t *origin, *status;
    double2 *ke;   // workspace (d_K, eta) per root (rebuilt by loewner)
    double2 *dz;   // workspace (d_i, zhat_i) per pole
    double *zhat, *bnorm;
};
// pack = false: the (d_K, eta) pairs were packed already (launch_pack_ke)
hipError_t launch_loewner(const VecArgs &a, int split, Queue *q, int grid, hipStream_t s,
                          bool pack = true);
hipError_t launch_pack_ke(const VecArgs &a, hipStream_t s);
hipError_t launch_bnorm(const VecArgs &a, int split, Queue *q, int grid, hipStream_t s);

struct ApplyArgs {
    const int64_t *off;
    const Tile *tiles;
    int ntiles;
    const double *d, *zhat, *bnorm, *eta;
    const int32_t *origin, *status;
    int trans;
    int m;
    const double *X;
    int64_t ldx;
    double *Y;
    int64_t ldy;
    int fuse_b;    // trans 1, MFMA, m < 16: form b with the kernel 1/t^2 on the weights
    double *bout;  // zhat^2 beside the m columns, write it here and scale by it
    unsigned long long *work;  // kernel timing on: algorithmic flops of the launch, (2m + 3)
                               // per Cauchy entry plus 2m per output row (set by launch_apply)
};
hipError_t launch_apply(const ApplyArgs &a, int use_mfma, Queue *q, int grid, hipStream_t s);

struct BwdArgs {
    const int64_t *off;
    const Tile *tiles;
    int ntiles;
    int nprob;
    const double *d, *z, *rho, *eta;
    const int32_t *origin, *status;
    const double *g_lam, *g_proj, *u;
    double *g_d, *g_z, *g_rho;
    double4 *pz;    // workspace (d_i, z_i, u_i, 0) per pole
    double4 *rk;    // workspace (d_K, eta, alpha, beta) per root
    double *gk;     // workspace gamma per root
};
hipError_t launch_backward(const BwdArgs &a, int split, int prob_first, int nprob, Queue *q1,
                           Queue *q2, int grid, hipStream_t s);

// deflation (deflate.hip)
hipError_t launch_deflate(const int64_t *off, int nprob, const double *d, const double *z,
                          const double *rho, double tau, double *dout, double *zout,
                          int32_t *perm, int32_t *rright, int32_t *rleft, double *rc, double *rs,
                          int32_t *kept, int32_t *status, double2 *val, int8_t *flag,
                          int max_n, int4 *seg_i, double2 *seg_d, hipStream_t s);
// segments per problem of the deflation scan (records seg_i, seg_d: nprob times this)
int deflate_segments(int max_n);
hipError_t launch_deflate_expand(const int64_t *off, int nprob, int64_t total, int m,
                                 const int32_t *perm, const int32_t *rright,
                                 const int32_t *rleft, const double *rc, const double *rs,
                                 int trans, const double *X, int64_t ldx, double *Y,
                                 int64_t ldy, double *T, hipStream_t s);
hipError_t launch_copy_rows(const int64_t *soff, const int64_t *doff, int nprob,
                            int64_t dtotal, int m, const int32_t *rows, const double *src,
                            int64_t lds, double *dst, int64_t ldd, const double *fill,
                            hipStream_t s);
}  // namespace sdc
#endif
