// Entry points built on the FFT product:
//   msb_apply / msb_apply_dinfl     f = A u (Sec. 3-4), or the a_k-derivative operator
//   msb_solve_static                static model eq. (mat:e2) by conjugate gradients,
//                                   FP64, FP32, or FP32 inside FP64 iterative refinement
//   msb_vv_init / msb_vv_run        dynamic model eq. (mat:e1) by velocity Verlet (Alg. 2)
//   msb_grad_infl                   adjoint gradient w.r.t. influence coefficients
//
// CG keeps every scalar on the device: each block that needs alpha or beta sums the
// per-block partial products itself in a fixed order, so there is no host round trip
// per iteration and results are bitwise reproducible.  Per-case flags stop converged
// cases of a batch while the others continue.  Blocks of iterations can be captured
// once into a hipGraph and replayed.
#include <chrono>
#include <mutex>
#include <cstring>
#include <cmath>
#include <cstdlib>

#include "fft_device.hpp"
#include "passes.hpp"

namespace msb {

constexpr int kT = 256;

// flags in SolverWs::done
enum : int { RUNNING = 0, CONVERGED = 1, BREAKDOWN = 2, NONFINITE = 3, SKIPPED = 4, CAPPED = 5 };

struct SolverWs {
    size_t nvec = 0;                 // B * d * N
    double *v64[6] = {};             // FP64 vectors
    float *v32[6] = {};              // FP32 vectors
    double *alt64[3] = {};           // fused CG: the second r, p, q (allocated on first use)
    float *alt32[3] = {};
    double *part_x = nullptr;        // [3][B * rows] x-inverse epilogue partials
    double *part_rr = nullptr;       // [2][B][tiles] true r.r partials (by iteration parity)
    double *part_aux = nullptr;      // [3][B][P] dot partials
    double *case4 = nullptr;         // [B][5] CG case sums (many tiles per case)
    double *part_rz = nullptr;       // [2][3][B * rows] preconditioned CG: r.z partials by parity
    double *part_adr = nullptr;      // [3][B * rows] dynamic relaxation: damping partials of the last force
    double *adr_D64 = nullptr;       // [slots][d][N] fictitious density
    float *adr_D32 = nullptr;
    int adr_slots = 0;
    int adr_prec = -1;               // precision of the last relaxation run (its partials), -1 none
    int adr_tiles = 0;               // x tiles per case its partials were written with
    bool adr_pending = false;        // restarted without an update: the next update is the first
    int64_t adr_version = -1;        // operator version D was built for
    double *thresh = nullptr;        // [B]
    double *scal = nullptr;          // [16][B] per-case scalars
    double *energy = nullptr;        // energies (device)
    size_t energy_cap = 0;
    int *done = nullptr;             // [2][B] flags by CG iteration parity; [0] is the final state
    int *iters = nullptr;            // [B]
    int *ecount = nullptr;           // energy counter
    double *h_scal = nullptr;        // pinned [16][B]
    int *h_int = nullptr;            // pinned [4][B]
    int P = 1;                       // vector-kernel blocks per case
    hipStream_t st = nullptr;        // internal stream (graph capture needs a non-null stream)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // captured blocks of CG iterations kept for later solves with the same arguments (the
    // inner solves of the refinement loop): key = every argument the iterations read
    struct CgGraph {
        std::vector<unsigned char> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    } graphs[2];
    int graph_next = 0;              // entry the next new graph replaces
};

static void drop_graph(SolverWs::CgGraph &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = SolverWs::CgGraph();
}

void solver_cache_free(msb_plan_s *p) {
    SolverWs *w = static_cast<SolverWs *>(p->solver_cache);
    if (!w) return;
    for (auto x : w->v64)
        if (x) (void)hipFree(x);
    for (auto x : w->v32)
        if (x) (void)hipFree(x);
    for (auto x : w->alt64)
        if (x) (void)hipFree(x);
    for (auto x : w->alt32)
        if (x) (void)hipFree(x);
    void *b[] = {w->part_x, w->part_rr, w->part_aux, w->case4, w->part_rz, w->part_adr, w->adr_D64, w->adr_D32,
                 w->thresh, w->scal, w->energy, w->done, w->iters, w->ecount};
    for (void *x : b)
        if (x) (void)hipFree(x);
    if (w->h_scal) (void)hipHostFree(w->h_scal);
    if (w->h_int) (void)hipHostFree(w->h_int);
    for (auto &g : w->graphs) drop_graph(g);
    if (w->ev_in) (void)hipEventDestroy(w->ev_in);
    if (w->ev_out) (void)hipEventDestroy(w->ev_out);
    if (w->st) (void)hipStreamDestroy(w->st);
    delete w;
    p->solver_cache = nullptr;
}

static msb_status alloc_ws(msb_plan_s *p, SolverWs *w);

// The plan's solver workspace, allocated on first use; a failed allocation frees the
// partial workspace (the next call starts over).
static msb_status get_ws(msb_plan_s *p, SolverWs *&out) {
    if (p->solver_cache) {
        out = static_cast<SolverWs *>(p->solver_cache);
        return MSB_OK;
    }
    SolverWs *w = new SolverWs();
    p->solver_cache = w;
    const msb_status s = alloc_ws(p, w);
    if (s != MSB_OK) {
        solver_cache_free(p);
        return s;
    }
    out = w;
    return MSB_OK;
}

static msb_status alloc_ws(msb_plan_s *p, SolverWs *w) {
    const int B = p->B;
    w->nvec = (size_t)B * p->dim * p->N;
    const size_t dn = (size_t)p->dim * p->N;
    w->P = (int)std::max<size_t>(1, std::min<size_t>(256, (dn + 4095) / 4096));
    for (auto &x : w->v64) MSB_HIP(hipMalloc(&x, sizeof(double) * w->nvec));
    for (auto &x : w->v32) MSB_HIP(hipMalloc(&x, sizeof(float) * w->nvec));
    MSB_HIP(hipMalloc(&w->part_x, sizeof(double) * 3 * (size_t)B * partial_slots(p)));
    // r.r partials by parity: x tiles of the prologue, or blocks of the fused CG step
    MSB_HIP(hipMalloc(&w->part_rr, sizeof(double) * 2 * (size_t)B * std::max<int64_t>(partial_slots(p), w->P)));
    MSB_HIP(hipMalloc(&w->part_aux, sizeof(double) * 3 * (size_t)B * w->P));
    MSB_HIP(hipMalloc(&w->case4, sizeof(double) * 5 * (size_t)B));
    MSB_HIP(hipMalloc(&w->part_rz, sizeof(double) * 6 * (size_t)B * rows_total(p)));
    MSB_HIP(hipMalloc(&w->thresh, sizeof(double) * B));
    MSB_HIP(hipMalloc(&w->scal, sizeof(double) * 16 * B));
    MSB_HIP(hipMalloc(&w->done, sizeof(int) * 2 * B));
    MSB_HIP(hipMalloc(&w->iters, sizeof(int) * B));
    MSB_HIP(hipMalloc(&w->ecount, sizeof(int)));
    MSB_HIP(hipHostMalloc(&w->h_scal, sizeof(double) * 16 * B));
    MSB_HIP(hipHostMalloc(&w->h_int, sizeof(int) * 4 * B));
    MSB_HIP(hipStreamCreateWithFlags(&w->st, hipStreamNonBlocking));
    MSB_HIP(hipEventCreateWithFlags(&w->ev_in, hipEventDisableTiming));
    MSB_HIP(hipEventCreateWithFlags(&w->ev_out, hipEventDisableTiming));
    return MSB_OK;
}

// Device buffer owned for the duration of a call (freed on every return path).
struct CallBuf {
    void *p = nullptr;
    ~CallBuf() {
        if (p) (void)hipFree(p);
    }
};

// ------------------------------------------------------------------ vector kernels
template <typename T> __global__ void k_fill(T *x, size_t n, T v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = v;
}

template <typename T> __global__ void k_fill_int(T *x, int n, T v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = v;
}

// dst = src on free DOFs (0 on constrained) when keep_fixed == 0;
// dst = src on constrained DOFs (0 on free) when keep_fixed == 1.
template <typename T>
__global__ void k_mask_copy(T *dst, const T *src, const uint8_t *fixed, size_t n, size_t dn, int keep_fixed) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const bool fx = fixed && fixed[i % dn];
        dst[i] = (fx == (keep_fixed != 0)) ? src[i] : T(0);
    }
}

// u_C = g_C (or 0)
template <typename T>
__global__ void k_set_fixed(T *u, const T *g, const uint8_t *fixed, size_t n, size_t dn) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (fixed[i % dn]) u[i] = g ? g[i] : T(0);
}

template <typename S, typename D> __global__ void k_cast(D *dst, const S *src, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (D)src[i];
}

// x64 += d (d FP32 or FP64)
template <typename S> __global__ void k_add_to(double *x, const S *d, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] += (double)d[i];
}

// per-case partial dot products x.y: grid B*P blocks, part[b*P + blk]
template <typename T>
__global__ __launch_bounds__(kT) void k_dot_parts(const T *x, const T *y, double *part, size_t dn, int P) {
    __shared__ double red[96];
    const int b = blockIdx.x / P, blk = blockIdx.x - b * P;
    const T *xb = x + (size_t)b * dn, *yb = y + (size_t)b * dn;
    double v[1] = {0.0};
    for (size_t i = (size_t)blk * kT + threadIdx.x; i < dn; i += (size_t)P * kT) v[0] += (double)xb[i] * (double)yb[i];
    block_sum<1>(v, red, threadIdx.x, kT);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// out[b] = scale * sum of part[b*stride .. b*stride + n)  (one block per case)
__global__ __launch_bounds__(kT) void k_case_sums(const double *part, int n, size_t stride, double *out, double scale) {
    __shared__ double red[96];
    const double s = block_sum_partials(part + (size_t)blockIdx.x * stride, n, red, threadIdx.x, kT);
    if (threadIdx.x == 0) out[blockIdx.x] = scale * s;
}

// CG start: thresh[b] = tol2 * (r.r)[b] (tol2_case[b] instead of tol2 when given);
// both parity slots of the flags (done[b], done[b + stride]): SKIPPED when skip[b] != 0,
// CONVERGED when r.r == 0, else RUNNING
__global__ void k_cg_setup(const double *rr_part, int P, double tol2, const double *tol2_case, double *thresh,
                           int *done, size_t stride, const int *skip, int *iters, int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    for (int i = 0; i < P; ++i) s += rr_part[(size_t)b * P + i];
    thresh[b] = (tol2_case ? tol2_case[b] : tol2) * s;
    const int f = (skip && skip[b]) ? SKIPPED : (s == 0.0 ? CONVERGED : RUNNING);
    done[b] = f;
    done[b + stride] = f;
    iters[b] = 0;
}

// a = (a + b)/rho on free DOFs, 0 on constrained
template <typename T>
__global__ void k_vv_accel(T *a, const T *bf, const uint8_t *fixed, size_t n, size_t dn, double rho) {
    const T ri = T(1.0 / rho);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const bool fx = fixed && fixed[i % dn];
        a[i] = fx ? T(0) : (a[i] + bf[i]) * ri;
    }
}

// H = rho V/2 sum v^2 - V/2 sum u.f - V sum b.u over all tiles of all cases
__global__ __launch_bounds__(kT) void k_energy(const double *part, int n, double rho, double V, double *energy, int *count) {
    __shared__ double red[96];
    const double uf = block_sum_partials(part, n, red, threadIdx.x, kT);
    const double vv = block_sum_partials(part + n, n, red, threadIdx.x, kT);
    const double bu = block_sum_partials(part + 2 * (size_t)n, n, red, threadIdx.x, kT);
    if (threadIdx.x == 0) {
        energy[*count] = 0.5 * rho * V * vv - 0.5 * V * uf - V * bu;
        *count += 1;
    }
}

static inline int grid_for(size_t n) { return (int)std::max<size_t>(1, std::min<size_t>(2048, (n + kT - 1) / kT)); }

// ------------------------------------------------------------------ helpers
template <typename T> struct Prec;
template <> struct Prec<double> { static constexpr msb_precision p = MSB_FP64; };
template <> struct Prec<float> { static constexpr msb_precision p = MSB_FP32; };

static msb_status check_plan(msb_plan_s *p) {
    MSB_CHECK(p, MSB_EINVAL, "null plan");
    int dev = -1;
    MSB_HIP(hipGetDevice(&dev));
    MSB_CHECK(dev == p->device, MSB_EINVAL, "plan was created on device %d, current is %d", p->device, dev);
    return MSB_OK;
}

template <typename T>
static msb_status product(msb_plan_s *p, const DeviceOp &op, const T *u, EndArgs<T> e, hipStream_t st) {
    PassArgs<T> a = pass_args<T>(p, op);
    e.pio = const_cast<T *>(u);
    if (!e.uin) e.uin = u;
    return launch_product<T>(a, e, st);
}

template <typename T> static EndArgs<T> end_args() {
    EndArgs<T> e;
    memset(&e, 0, sizeof(e));
    e.sign = 1.0;
    e.rho = 1.0;
    return e;
}

// ------------------------------------------------------------------ conjugate gradients
template <typename T> static T **alt_vectors(SolverWs *w);
template <> double **alt_vectors<double>(SolverWs *w) { return w->alt64; }
template <> float **alt_vectors<float>(SolverWs *w) { return w->alt32; }

template <typename T> struct Cg {
    msb_plan_s *p;
    SolverWs *w;
    hipStream_t st;
    T *x, *r, *pv, *q;
    PassArgs<T> pa;
    int tpc;
    const double *prev_rr;   // r.r partials before a residual replacement (first beta), or null
    // fused steps: iteration it >= 1 reads r, p, q of set (it + 1) & 1 and writes set it & 1
    // (set 0: r, pv, q; set 1: r1, p1, q1); r.r partials per block, parity stride B rr_slots
    bool fused = false;
    T *r1 = nullptr, *p1 = nullptr, *q1 = nullptr;
    int rr_slots = 0;
};

// r.r partials of a CG run on a plan: per case count and parity stride (the x tiles of
// the prologue, or the product's blocks when the steps are fused into the tiled kernel).
template <typename T> static bool cg_fusable(const PassArgs<T> &pa) {
    // a register kernel with the CG-epilogue form (frame 16, and 32 and 64 in FP32), one block
    // per workgroup, and no term that reads the transformed vector off the block's own nodes
    // (broken bonds, surface correction): the patch forms the new p itself
    const bool form = pa.tl == 16 || ((pa.tl == 32 || pa.tl == 64) && sizeof(T) == 4);
    return form && pa.treg && pa.tper == 1 && pa.corr && !pa.br_row_ptr && !pa.nu;
}
struct RrLayout {
    int per_case;   // partials per case
    size_t stride;  // between the two parity arrays
};
template <typename T> static RrLayout cg_rr_layout(const msb_plan_s *p, const PassArgs<T> &pa) {
    const int tpc = x_tiles_per_case(p, pa.F);
    if (!cg_fusable(pa)) return RrLayout{tpc, (size_t)p->B * tpc};
    return RrLayout{pa.ept, (size_t)p->B * std::max(tpc, pa.ept)};
}

// Per-case sums of the tile partials the next CG step needs, one block per case
// (src[k] + b tiles: the K arrays in the order the prologue reduces them).  Used when a
// case has many tiles: every x-forward block would otherwise re-reduce all of its
// case's partials.
struct SumSrc {
    const double *p[5];
    int n[5];   // partials per case of each array
};
// 8 waves: a case's partials (a few thousand per array at most tiles) are loaded in one or
// two rounds of independent loads, the reduction being latency-bound (measured against 4 and
// 16 waves: plate512 CG 2.5% faster than with 16)
constexpr int kSumT = 512;
template <int K> __global__ __launch_bounds__(kSumT) void k_cg_sums(SumSrc src, double *out) {
    __shared__ double red[96];
    const int b = blockIdx.x;
    const double *parts[K];
    int cnt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        parts[k] = src.p[k] + (size_t)b * src.n[k];
        cnt[k] = src.n[k];
    }
    double sums[K];
    block_sum_partials_k<K>(parts, cnt, sums, red, threadIdx.x, blockDim.x);
    if (threadIdx.x == 0) {
        for (int k = 0; k < K; ++k) out[(size_t)b * K + k] = sums[k];
    }
}

// Tiles per case above which the per-case sums come from k_cg_sums.
constexpr int kFusedReduceMaxTiles = 1024;

// The per-case sums of one plan-group member for one CG slot: K arrays of partials (p[k] +
// case * n[k]), results to out[case * K + k]; out null: the member reduces in its prologue
// (few tiles per case), as the plan alone does.
struct GroupSum {
    const double *p[5];
    int n[5];
    double *out;
};

// k_cg_sums over the cases of several members: one workgroup per case; cstart[] holds the
// members' case offsets (cstart[n] = the cases of the launch).
template <int K>
__global__ __launch_bounds__(kSumT) void k_group_sums(const GroupSum *__restrict__ S, const int *__restrict__ cstart,
                                                      int n) {
    __shared__ double red[96];
    const int c = blockIdx.x;
    const int j = group_member(cstart, n, c);
    const GroupSum &s = S[j];
    if (!s.out) return;   // uniform over the workgroup
    const int b = c - cstart[j];
    const double *parts[K];
    int cnt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        parts[k] = s.p[k] + (size_t)b * s.n[k];
        cnt[k] = s.n[k];
    }
    double sums[K];
    block_sum_partials_k<K>(parts, cnt, sums, red, threadIdx.x, blockDim.x);
    if (threadIdx.x == 0) {
        for (int k = 0; k < K; ++k) s.out[(size_t)b * K + k] = sums[k];
    }
}

// One CG iteration = one product chain.  The x-forward prologue applies the
// previous iteration's update (x += alpha p, r -= alpha q, alpha and beta from the
// previous partial sums) and forms p = r + beta p; the x-inverse epilogue forms
// q = K p and the partials p.q, r.q, q.q.  No separate vector kernel.
template <typename T> static msb_status cg_iteration(Cg<T> &c, int it, bool update_only = false) {
    msb_plan_s *p = c.p;
    SolverWs *w = c.w;
    const int B = p->B;
    const size_t nt = (size_t)B * (c.fused ? c.rr_slots : c.tpc);
    const int ept = c.pa.ept;                 // epilogue partials per case (x-inverse or tiles)
    const size_t ne = (size_t)B * ept;
    if (c.fused && it > 0) {
        // one launch: the previous step's update applied on the patches, then q = K p
        T *rs[2] = {c.r, c.r1}, *ps[2] = {c.pv, c.p1}, *qs[2] = {c.q, c.q1};
        const int rd = (it + 1) & 1, wr = it & 1;
        const double *rr_prev = w->part_rr + (size_t)rd * nt;
        const SumSrc src{{rr_prev, w->part_x, w->part_x + ne, w->part_x + 2 * ne, nullptr}, {ept, ept, ept, ept, 0}};
        hipLaunchKernelGGL(k_cg_sums<4>, dim3(B), dim3(kSumT), 0, c.st, src, w->case4);
        EndArgs<T> e = end_args<T>();
        e.pro = PRO_NONE;
        e.cg_fused = 1;
        e.pio = ps[rd];
        e.cr = rs[rd];
        e.cq = qs[rd];
        e.cx = c.x;
        e.p_new = ps[wr];
        e.r_new = rs[wr];
        e.case4 = w->case4;
        e.rr_out = w->part_rr + (size_t)wr * nt;
        e.update_only = update_only;
        e.iters = w->iters;
        e.done_prev = w->done + (size_t)rd * B;
        e.done_rw = w->done + (size_t)wr * B;
        e.thresh = w->thresh;
        e.epi = EPI_CG_Q;
        e.uin = ps[wr];
        e.out = qs[wr];
        e.rhs = rs[wr];
        e.part = w->part_x;
        return launch_product<T>(c.pa, e, c.st);
    }
    EndArgs<T> e = end_args<T>();
    e.pro = PRO_CG_P;
    e.pio = c.pv;
    e.cx = c.x;
    e.cr = c.r;
    e.cq = c.q;
    e.cg3 = w->part_x;
    e.n_cg3 = ept;
    e.s_cg3 = ne;
    e.rr_prev = w->part_rr + (size_t)((it + 1) & 1) * nt;
    e.rr_out = w->part_rr + (size_t)(it & 1) * nt;
    e.first = it == 0;
    e.update_only = update_only;
    if (it > 0 && std::max(c.tpc, ept) > kFusedReduceMaxTiles) {
        const SumSrc src{{e.rr_prev, e.cg3, e.cg3 + ne, e.cg3 + 2 * ne, nullptr}, {c.tpc, ept, ept, ept, 0}};
        hipLaunchKernelGGL(k_cg_sums<4>, dim3(B), dim3(kSumT), 0, c.st, src, w->case4);
        e.case4 = w->case4;
    }
    e.iters = w->iters;
    if (it == 0 && c.prev_rr) {   // continuation after a residual replacement
        e.beta_num = w->part_aux;
        e.n_num = w->P;
        e.beta_den = c.prev_rr;
        e.n_den = c.fused ? ept : c.tpc;
    }
    e.rr_tiles = c.fused;   // the next (fused) step reads r.r partials per block
    e.done_prev = w->done + (size_t)((it + 1) & 1) * B;
    e.case_done = w->done + (size_t)(it & 1) * B;
    e.done_rw = w->done + (size_t)(it & 1) * B;
    e.thresh = w->thresh;
    e.epi = EPI_CG_Q;
    e.uin = c.pv;
    e.out = c.q;
    e.rhs = c.r;
    e.part = w->part_x;
    return launch_product<T>(c.pa, e, c.st);
}

// Iterations between host checks of the per-case done flags when no graph is used.
constexpr int kPollIterations = 32;
// FP64 solves: restarts of CG from the FP64 residual when the recurrence met the
// tolerance but the residual b' - K u does not.
constexpr int kPolish = 4;

// Argument bytes of a captured block of iterations (the cache key of its graph).
struct GraphKey {
    std::vector<unsigned char> b;
    template <typename V> void add(const V &v) {
        const unsigned char *q = reinterpret_cast<const unsigned char *>(&v);
        b.insert(b.end(), q, q + sizeof(V));
    }
};

// Run CG iterations iter(it, update_only) from the prepared state (vectors, partials,
// thresholds and both parity slots of the flags set).  Stops when every case has a
// flag or after maxit iterations; the final flags end in slot 0.  Blocks of iterations
// 1 .. (every block starts at an odd iteration, so all are alike) run as one hipGraph
// when graph_block > 0; with a key, the graph is kept in the workspace and replayed by
// later calls with the same key (no new capture per inner solve).
template <typename It>
static msb_status run_iterations(SolverWs *w, int B, hipStream_t st, It iter, int maxit, int graph_block,
                                 int *it_out, GraphKey *key = nullptr) {
    int it = 0;
    MSB_TRY(iter(0, false));
    it = 1;
    const int poll = graph_block > 0 ? graph_block : kPollIterations;
    const int block = poll + (poll & 1);   // even: keeps the partial-sum parity of replays fixed
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    bool cached = false;                   // exec belongs to the workspace cache
    if (key && graph_block > 0) {
        key->add(block);
        for (auto &g : w->graphs)
            if (g.exec && g.key == key->b) {
                exec = g.exec;
                cached = true;
            }
    }
    msb_status s = MSB_OK;
    while (it < maxit && s == MSB_OK) {
        MSB_HIP(hipMemcpyAsync(w->h_int, w->done + (size_t)((it - 1) & 1) * B, sizeof(int) * B,
                               hipMemcpyDeviceToHost, st));
        MSB_HIP(hipStreamSynchronize(st));
        bool all = true;
        for (int b = 0; b < B; ++b) all = all && w->h_int[b] != RUNNING;
        if (all) break;
        const int k = std::min(block, maxit - it);
        if (graph_block > 0 && k == block) {
            if (!exec) {
                MSB_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                for (int j = 0; j < block && s == MSB_OK; ++j) s = iter(it + j, false);
                hipError_t e1 = hipStreamEndCapture(st, &graph);
                if (s != MSB_OK) break;
                MSB_HIP(e1);
                MSB_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
                if (key) {   // keep it: replaces the older entry
                    SolverWs::CgGraph &g = w->graphs[w->graph_next];
                    w->graph_next = (w->graph_next + 1) % 2;
                    drop_graph(g);
                    g.key = key->b;
                    g.graph = graph;
                    g.exec = exec;
                    graph = nullptr;
                    cached = true;
                }
            }
            MSB_HIP(hipGraphLaunch(exec, st));
        } else {
            for (int j = 0; j < k && s == MSB_OK; ++j) s = iter(it + j, false);
        }
        it += k;
    }
    if (exec && !cached) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    // iteration cap: apply the pending update of the cases still running
    if (s == MSB_OK) s = iter(it, true);
    if (s == MSB_OK && (it & 1))   // the final flags into slot 0
        MSB_HIP(hipMemcpyAsync(w->done, w->done + B, sizeof(int) * B, hipMemcpyDeviceToDevice, st));
    *it_out = it;
    return s;
}

template <typename T> static msb_status run_cg(Cg<T> &c, int maxit, int graph_block, int *it_out) {
    auto iter = [&c](int it, bool upd) { return cg_iteration(c, it, upd); };
    // everything iterations >= 1 read (c.prev_rr only enters iteration 0)
    GraphKey key;
    key.add((int)sizeof(T));
    key.add(0);
    key.add(c.pa);
    key.add(c.x), key.add(c.r), key.add(c.pv), key.add(c.q), key.add(c.tpc), key.add(c.st);
    key.add(c.fused), key.add(c.r1), key.add(c.p1), key.add(c.q1), key.add(c.rr_slots);
    return run_iterations(c.w, c.p->B, c.st, iter, maxit, graph_block, it_out, &key);
}

// Denominator of the first beta after a residual replacement (reliable update): the
// partials of the step that formed the search direction the run ended with.  Iteration
// k >= 1 applies update k, so after K updates of case b that direction was formed at
// iteration K - 1, whose partials sit in parity slot (K - 1) & 1 (part + slot * pstride):
// r.r for CG, r.z for preconditioned CG.  No update (K = 0): zeros (beta = 0, a restart).
__global__ void k_save_last(const double *part, size_t pstride, const int *iters, int P, double *dst) {
    const int b = blockIdx.x;
    const int K = iters[b];
    const double *src = part + (size_t)((K + 1) & 1) * pstride + (size_t)b * P;
    for (int i = threadIdx.x; i < P; i += blockDim.x) dst[(size_t)b * P + i] = K > 0 ? src[i] : 0.0;
}

// Prepare and run CG on K d = rhs (rhs already masked); x0 = 0.  With prev_rr the
// search direction pv is kept (reliable update after a residual replacement) and the
// first beta is (new r.r) / prev_rr; otherwise pv starts at 0 (plain restart).
template <typename T>
static msb_status cg_solve(msb_plan_s *p, SolverWs *w, hipStream_t st, const T *rhs, T *x, T *r, T *pv,
                           T *q, double tol, int maxit, int graph_block, const int *skip,
                           const double *prev_rr = nullptr, int *iters_out = nullptr,
                           const double *tol2_case = nullptr) {
    const size_t n = w->nvec;
    const int B = p->B, P = w->P;
    Cg<T> c{p, w, st, x, r, pv, q, pass_args<T>(p, p->op), 0, prev_rr};
    c.tpc = x_tiles_per_case(p, c.pa.F);
    if (cg_fusable(c.pa)) {
        T **alt = alt_vectors<T>(w);
        for (int k = 0; k < 3; ++k)
            if (!alt[k]) MSB_HIP(hipMalloc(&alt[k], sizeof(T) * n));
        c.fused = true;
        c.r1 = alt[0], c.p1 = alt[1], c.q1 = alt[2];
        c.rr_slots = std::max(c.tpc, c.pa.ept);
    }
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kT), 0, st, x, n, T(0));
    if (!prev_rr) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kT), 0, st, pv, n, T(0));
    hipLaunchKernelGGL((k_cast<T, T>), dim3(grid_for(n)), dim3(kT), 0, st, r, rhs, n);
    hipLaunchKernelGGL(k_dot_parts<T>, dim3(B * P), dim3(kT), 0, st, (const T *)r, (const T *)r, w->part_aux,
                       (size_t)p->dim * p->N, P);
    hipLaunchKernelGGL(k_cg_setup, dim3((B + 63) / 64), dim3(64), 0, st, (const double *)w->part_aux, P, tol * tol,
                       tol2_case, w->thresh, w->done, (size_t)B, skip, w->iters, B);
    MSB_HIP(hipGetLastError());
    int it = 0;
    msb_status r0 = run_cg(c, maxit, graph_block, &it);
    if (r0 == MSB_OK && c.fused && (it & 1)) {
        // the last step wrote set 1: r and the search direction back to the caller's vectors
        MSB_HIP(hipMemcpyAsync(r, c.r1, sizeof(T) * n, hipMemcpyDeviceToDevice, st));
        MSB_HIP(hipMemcpyAsync(pv, c.p1, sizeof(T) * n, hipMemcpyDeviceToDevice, st));
    }
    if (iters_out) *iters_out = it;
    return r0;
}

// ------------------------------------------------------------------ preconditioned CG
// A circulant preconditioner (the introduction cites preconditioned fast Toeplitz
// methods as prior work; it is not part of MSBFM itself): C^{-1} with symbol
// (Khat(k) + s I)^{-1} per frequency of the padded grid, applied by the same product
// chain without the boundary corrections, so z = Pi_F E^T C^{-1} E Pi_F r (E: zero
// padding to the transform lengths) is symmetric positive definite on the free DOFs.
// Built on first use, dropped with the operator.
static msb_status ensure_pre(msb_plan_s *p) {
    if (p->pre.count > 0) return MSB_OK;
    return build_preconditioner(p);
}

template <typename T> struct Pcg {
    msb_plan_s *p;
    SolverWs *w;
    hipStream_t st;
    T *x, *r, *pv, *q, *z;
    PassArgs<T> pa;   // stiffness product
    PassArgs<T> pp;   // preconditioner product (spectral symbol only)
    int tpc;
    const double *prev_rz;   // r.z partials before a residual replacement (first beta), or null
    // fused stiffness steps (iterations >= 1): p alternates between pv (set 0) and p1 (set 1);
    // iteration it reads set (it + 1) & 1 and writes set it & 1
    bool fused = false;
    T *p1 = nullptr;
};

// One preconditioned CG iteration = two product chains.
//   P chain: the x-forward applies the previous update (x += alpha p, r -= alpha q with
//            alpha = r.z / p.q) and transforms r; the x-inverse forms z = C^{-1} r and
//            the partials r.z.
//   A chain: the x-forward forms p = z + beta p (beta = r.z / previous r.z) and
//            transforms p; the x-inverse forms q = K p and the partials p.q, r.q, q.q.
// Convergence is tested on the true r.r (summed in the P chain's x-forward) against the
// same threshold as plain CG.
template <typename T> static msb_status pcg_iteration(Pcg<T> &c, int it, bool update_only) {
    msb_plan_s *p = c.p;
    SolverWs *w = c.w;
    const int B = p->B;
    const size_t nt = (size_t)B * c.tpc;
    const int ept = c.pa.ept;                 // the stiffness chain's epilogue partials per case
    const size_t ne = (size_t)B * ept;
    const int cur = it & 1, prv = (it + 1) & 1;
    const bool reduce = it > 0 && std::max(c.tpc, ept) > kFusedReduceMaxTiles;
    T *ps[2] = {c.pv, c.fused ? c.p1 : c.pv};
    {
        EndArgs<T> e = end_args<T>();
        e.pro = PRO_PCG_R;
        e.pr = ps[prv];   // the search direction of the previous iteration
        e.cx = c.x;
        e.cr = c.r;
        e.cq = c.q;
        e.cg3 = w->part_x;
        e.n_cg3 = ept;
        e.s_cg3 = ne;
        e.rr_prev = w->part_rr + (size_t)prv * nt;
        e.rr_out = w->part_rr + (size_t)cur * nt;
        e.rz_k = w->part_rz + (size_t)prv * 3 * nt;
        e.first = it == 0;
        e.update_only = update_only;
        if (reduce) {
            const SumSrc src{{e.rr_prev, e.rz_k, e.cg3, e.cg3 + ne, e.cg3 + 2 * ne}, {c.tpc, c.tpc, ept, ept, ept}};
            hipLaunchKernelGGL(k_cg_sums<5>, dim3(B), dim3(kSumT), 0, c.st, src, w->case4);
            e.case4 = w->case4;
        }
        e.iters = w->iters;
        e.done_prev = w->done + (size_t)prv * B;
        e.case_done = w->done + (size_t)cur * B;
        e.done_rw = w->done + (size_t)cur * B;
        e.thresh = w->thresh;
        e.epi = EPI_PCG_Z;
        e.uin = c.r;
        e.out = c.z;
        e.sign = 1.0;
        e.part = w->part_rz + (size_t)cur * 3 * nt;
        MSB_TRY(launch_product<T>(c.pp, e, c.st));
    }
    if (update_only) return MSB_OK;
    if (c.fused && it > 0) {
        // one launch: p = z + beta p on the patches (beta from the case sums), then q = K p
        const SumSrc src{{w->part_rz + (size_t)cur * 3 * nt, w->part_rz + (size_t)prv * 3 * nt, nullptr, nullptr,
                          nullptr},
                         {c.tpc, c.tpc, 0, 0, 0}};
        hipLaunchKernelGGL(k_cg_sums<2>, dim3(B), dim3(kSumT), 0, c.st, src, w->case4);
        EndArgs<T> e = end_args<T>();
        e.pro = PRO_NONE;
        e.cg_fused = 2;
        e.pr = c.z;
        e.pio = ps[prv];
        e.p_new = ps[cur];
        e.case4 = w->case4;
        e.case_done = w->done + (size_t)cur * B;
        e.epi = EPI_CG_Q;
        e.uin = ps[cur];
        e.out = c.q;
        e.rhs = c.r;
        e.part = w->part_x;
        return launch_product<T>(c.pa, e, c.st);
    }
    EndArgs<T> e = end_args<T>();
    e.pro = PRO_PCG_P;
    e.pr = c.z;
    e.pio = c.pv;
    e.rz_k = w->part_rz + (size_t)cur * 3 * nt;
    e.rz_km1 = w->part_rz + (size_t)prv * 3 * nt;
    e.first = it == 0;
    if (it == 0 && c.prev_rz) {   // continuation: p = z + (r.z / previous r.z) p with the kept p
        e.first = false;
        e.rz_km1 = c.prev_rz;
    }
    if (reduce) {
        const SumSrc src{{e.rz_k, e.rz_km1, nullptr, nullptr, nullptr}, {c.tpc, c.tpc, 0, 0, 0}};
        hipLaunchKernelGGL(k_cg_sums<2>, dim3(B), dim3(kSumT), 0, c.st, src, w->case4);
        e.case4 = w->case4;
    }
    e.case_done = w->done + (size_t)cur * B;
    e.epi = EPI_CG_Q;
    e.uin = c.pv;
    e.out = c.q;
    e.rhs = c.r;
    e.part = w->part_x;
    return launch_product<T>(c.pa, e, c.st);
}

// Preconditioned CG on K d = rhs (rhs already masked), x0 = 0, with the same flags,
// thresholds and iteration counters as cg_solve.  With prev_rz the search direction pv
// is kept (reliable update) and the first beta is (new r.z) / prev_rz.
template <typename T>
static msb_status pcg_solve(msb_plan_s *p, SolverWs *w, hipStream_t st, const T *rhs, T *x, T *r, T *pv, T *q,
                            T *z, double tol, int maxit, int graph_block, const int *skip, int *iters_out = nullptr,
                            const double *tol2_case = nullptr, const double *prev_rz = nullptr) {
    MSB_TRY(ensure_pre(p));
    const size_t n = w->nvec;
    const int B = p->B, P = w->P;
    Pcg<T> c{p, w, st, x, r, pv, q, z, pass_args<T>(p, p->op), pass_args<T>(p, p->pre), 0, prev_rz};
    c.pp.corr = 0;
    c.tpc = x_tiles_per_case(p, c.pa.F);
    if (cg_fusable(c.pa)) {
        T **alt = alt_vectors<T>(w);
        if (!alt[1]) MSB_HIP(hipMalloc(&alt[1], sizeof(T) * n));
        c.fused = true;
        c.p1 = alt[1];
    }
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kT), 0, st, x, n, T(0));
    if (!prev_rz) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kT), 0, st, pv, n, T(0));
    hipLaunchKernelGGL((k_cast<T, T>), dim3(grid_for(n)), dim3(kT), 0, st, r, rhs, n);
    hipLaunchKernelGGL(k_dot_parts<T>, dim3(B * P), dim3(kT), 0, st, (const T *)r, (const T *)r, w->part_aux,
                       (size_t)p->dim * p->N, P);
    hipLaunchKernelGGL(k_cg_setup, dim3((B + 63) / 64), dim3(64), 0, st, (const double *)w->part_aux, P, tol * tol,
                       tol2_case, w->thresh, w->done, (size_t)B, skip, w->iters, B);
    MSB_HIP(hipGetLastError());
    int it = 0;
    auto iter = [&c](int k, bool upd) { return pcg_iteration(c, k, upd); };
    GraphKey key;   // everything iterations >= 1 read (c.prev_rz only enters iteration 0)
    key.add((int)sizeof(T));
    key.add(1);
    key.add(c.pa), key.add(c.pp);
    key.add(c.x), key.add(c.r), key.add(c.pv), key.add(c.q), key.add(c.z), key.add(c.tpc), key.add(c.st);
    key.add(c.fused), key.add(c.p1);
    msb_status r0 = run_iterations(w, B, st, iter, maxit, graph_block, &it, &key);
    // the last stiffness step (iteration it - 1; iteration it updated only) wrote set 1: the
    // search direction back to pv
    if (r0 == MSB_OK && c.fused && it >= 1 && ((it - 1) & 1))
        MSB_HIP(hipMemcpyAsync(pv, c.p1, sizeof(T) * n, hipMemcpyDeviceToDevice, st));
    if (iters_out) *iters_out = it;
    return r0;
}

// per-case ||rhs + A x||^2 on free DOFs into w->scal[slot*B + b], residual vector into out
static msb_status true_residual(msb_plan_s *p, SolverWs *w, hipStream_t st, const double *x, const double *rhs,
                                double *out, int slot) {
    EndArgs<double> e = end_args<double>();
    e.epi = EPI_RESID;
    e.rhs = rhs;
    e.out = out;
    e.part = w->part_x;
    MSB_TRY(product<double>(p, p->op, x, e, st));
    const int ept = pass_args<double>(p, p->op).ept;
    hipLaunchKernelGGL(k_case_sums, dim3(p->B), dim3(kT), 0, st, (const double *)w->part_x, ept, (size_t)ept,
                       w->scal + (size_t)slot * p->B, 1.0);
    MSB_HIP(hipGetLastError());
    return MSB_OK;
}

static msb_status fetch_scal(SolverWs *w, hipStream_t st, int nslots, int B) {
    MSB_HIP(hipMemcpyAsync(w->h_scal, w->scal, sizeof(double) * nslots * B, hipMemcpyDeviceToHost, st));
    MSB_HIP(hipMemcpyAsync(w->h_int, w->done, sizeof(int) * B, hipMemcpyDeviceToHost, st));
    MSB_HIP(hipMemcpyAsync(w->h_int + B, w->iters, sizeof(int) * B, hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    return MSB_OK;
}

static msb_status flag_status(int f) {
    switch (f) {
        case CONVERGED: case SKIPPED: return MSB_OK;
        case BREAKDOWN: return MSB_ENOTSPD;
        case NONFINITE: return MSB_ENOTSPD;
        default: return MSB_ENOCONV;
    }
}

}  // namespace msb

using namespace msb;

// ---------------------------------------------------------------------------- apply
extern "C" msb_status msb_apply(msb_plan p, msb_precision prec, const void *u, void *f, void *stream) {
    MSB_TRY(check_plan(p));
    MSB_CHECK(u && f, MSB_EINVAL, "null vector");
    MSB_CHECK(u != f, MSB_EINVAL, "u and f must not overlap");
    hipStream_t st = (hipStream_t)stream;
    if (prec == MSB_FP64) {
        EndArgs<double> e = end_args<double>();
        e.epi = EPI_APPLY;
        e.out = (double *)f;
        return product<double>(p, p->op, (const double *)u, e, st);
    }
    MSB_CHECK(prec == MSB_FP32, MSB_EINVAL, "apply precision must be MSB_FP64 or MSB_FP32");
    EndArgs<float> e = end_args<float>();
    e.epi = EPI_APPLY;
    e.out = (float *)f;
    return product<float>(p, p->op, (const float *)u, e, st);
}

template <typename T> static msb_status apply_pre_t(msb_plan_s *p, const T *r, T *z, hipStream_t st) {
    MSB_TRY(ensure_pre(p));
    PassArgs<T> a = pass_args<T>(p, p->pre);
    a.corr = 0;
    EndArgs<T> e = end_args<T>();
    e.epi = EPI_APPLY;
    e.pio = const_cast<T *>(r);
    e.uin = r;
    e.out = z;
    return launch_product<T>(a, e, st);
}

extern "C" msb_status msb_apply_precond(msb_plan p, msb_precision prec, const void *r, void *z, void *stream) {
    MSB_TRY(check_plan(p));
    MSB_CHECK(r && z, MSB_EINVAL, "null vector");
    MSB_CHECK(r != z, MSB_EINVAL, "r and z must not overlap");
    hipStream_t st = (hipStream_t)stream;
    if (prec == MSB_FP64) return apply_pre_t<double>(p, (const double *)r, (double *)z, st);
    MSB_CHECK(prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    return apply_pre_t<float>(p, (const float *)r, (float *)z, st);
}

static msb_status ensure_dop(msb_plan_s *p, int k) {
    if ((int)p->dop.size() <= k) p->dop.resize(k + 1);
    DeviceOp &op = p->dop[k];
    if (op.count) return MSB_OK;
    std::vector<double> e(k + 1, 0.0);
    e[k] = 1.0;
    MSB_TRY(alloc_operator(p, op, 1));
    MSB_TRY(fill_operator(p, e, op, 0));
    return ensure_tiles(p);
}

extern "C" msb_status msb_apply_dinfl(msb_plan p, int k, const double *u, double *f, void *stream) {
    MSB_TRY(check_plan(p));
    MSB_CHECK(u && f && u != f, MSB_EINVAL, "bad vectors");
    MSB_CHECK(k >= 0 && k < 8, MSB_EINVAL, "k must be in [0, 8)");
    MSB_TRY(ensure_dop(p, k));
    EndArgs<double> e = end_args<double>();
    e.epi = EPI_APPLY;
    e.out = f;
    return product<double>(p, p->dop[k], u, e, (hipStream_t)stream);
}

template <typename T>
static msb_status profile_t(msb_plan_s *p, const T *u, T *f, int nrep, double *ms, int *npass, hipStream_t st) {
    // each pass launched nrep times back to back between two events: the mean kernel
    // duration of a launch in a stream of launches; then one plain product for f
    const int np = n_passes(pass_args<T>(p, p->op));
    std::vector<hipEvent_t> ev((size_t)(np + 1), nullptr);
    msb_status s = MSB_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) s = MSB_EDEVICE;
    EndArgs<T> e = end_args<T>();
    e.epi = EPI_APPLY;
    e.out = f;
    PassArgs<T> a = pass_args<T>(p, p->op);
    e.pio = const_cast<T *>(u);
    e.uin = u;
    if (s == MSB_OK) s = launch_product<T>(a, e, st, ev.data(), nrep);
    if (s == MSB_OK) s = launch_product<T>(a, e, st);
    if (s == MSB_OK && hipStreamSynchronize(st) != hipSuccess) s = MSB_EDEVICE;
    for (int i = 0; i < np && s == MSB_OK; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) s = MSB_EDEVICE;
        ms[i] = (double)t / nrep;
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    *npass = np;
    if (s != MSB_OK) set_error("event timing failed");
    return s;
}

extern "C" msb_status msb_profile_apply(msb_plan p, msb_precision prec, const void *u, void *f, int nrep,
                                        double *ms, int *npass, void *stream) {
    MSB_TRY(check_plan(p));
    MSB_CHECK(u && f && u != f && ms && npass && nrep > 0, MSB_EINVAL, "bad arguments");
    if (prec == MSB_FP64)
        return profile_t<double>(p, (const double *)u, (double *)f, nrep, ms, npass, (hipStream_t)stream);
    MSB_CHECK(prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    return profile_t<float>(p, (const float *)u, (float *)f, nrep, ms, npass, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------- static solve
extern "C" msb_status msb_solve_static(msb_plan p, msb_precision prec, const double *b, const double *g,
                                       double *u, const msb_solve_opts *opts, msb_solve_info *info,
                                       void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    MSB_TRY(check_plan(p));
    MSB_CHECK(b && u && opts && info, MSB_EINVAL, "null argument");
    MSB_CHECK(b != u && g != u, MSB_EINVAL, "u must not alias b or g");
    MSB_CHECK(opts->tol > 0 && opts->tol < 1 && opts->maxit > 0, MSB_EINVAL, "need 0 < tol < 1 and maxit > 0");
    MSB_CHECK(prec == MSB_FP64 || prec == MSB_FP32 || prec == MSB_FP32_REFINED, MSB_EINVAL, "bad precision");
    MSB_CHECK(opts->graph_block >= 0 && opts->graph_block <= 4096, MSB_EINVAL, "graph_block out of range");
    MSB_CHECK(opts->precond == 0 || opts->precond == 1, MSB_EINVAL, "precond must be 0 or 1");
    MSB_CHECK(!p->nu64, MSB_EUNSUPPORTED, "the surface-corrected operator is not symmetric: no CG solve");
    const bool pre = opts->precond != 0;
    SolverWs *w = nullptr;
    MSB_TRY(get_ws(p, w));
    const int B = p->B;
    const size_t n = w->nvec, dn = (size_t)p->dim * p->N;
    hipStream_t user = (hipStream_t)stream;
    hipStream_t st = w->st;
    MSB_HIP(hipEventRecord(w->ev_in, user));
    MSB_HIP(hipStreamWaitEvent(st, w->ev_in, 0));
    const int gb = opts->graph_block;

    double *bp = w->v64[0], *tmp = w->v64[1];
    // lifted right-hand side b' = b_F - K_FC g_C = (b + A g~)_F, g~ = g on Omega_c, 0 elsewhere
    if (g && p->fixed) {
        hipLaunchKernelGGL(k_mask_copy<double>, dim3(grid_for(n)), dim3(kT), 0, st, tmp, g, (const uint8_t *)p->fixed, n, dn, 1);
        EndArgs<double> e = end_args<double>();
        e.epi = EPI_RESID;
        e.rhs = b;
        e.out = bp;
        MSB_TRY(product<double>(p, p->op, tmp, e, st));
    } else {
        hipLaunchKernelGGL(k_mask_copy<double>, dim3(grid_for(n)), dim3(kT), 0, st, bp, b, (const uint8_t *)p->fixed, n, dn, 0);
    }
    hipLaunchKernelGGL(k_dot_parts<double>, dim3(B * w->P), dim3(kT), 0, st, (const double *)bp, (const double *)bp,
                       w->part_aux, dn, w->P);
    hipLaunchKernelGGL(k_case_sums, dim3(B), dim3(kT), 0, st, (const double *)w->part_aux, w->P, (size_t)w->P, w->scal, 1.0);
    MSB_HIP(hipGetLastError());
    MSB_TRY(fetch_scal(w, st, 1, B));
    std::vector<double> bb(w->h_scal, w->h_scal + B);
    for (int c = 0; c < B; ++c)
        MSB_CHECK(std::isfinite(bb[c]), MSB_EINVAL, "case %d: right-hand side (or lift) is not finite", c);

    std::vector<int> outer(B, 0), inner(B, 0), fl(B, RUNNING);
    std::vector<double> rel(B, 0.0);
    msb_status result = MSB_OK;

    if (prec == MSB_FP64 || prec == MSB_FP32) {
        if (prec == MSB_FP64) {
            if (pre)
                MSB_TRY(pcg_solve<double>(p, w, st, bp, u, w->v64[2], w->v64[3], w->v64[4], w->v64[5], opts->tol,
                                          opts->maxit, gb, nullptr));
            else
                MSB_TRY(cg_solve<double>(p, w, st, bp, u, w->v64[2], w->v64[3], w->v64[4], opts->tol, opts->maxit, gb,
                                         nullptr));
        } else {
            float *b32 = w->v32[0], *x32 = w->v32[1];
            hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(kT), 0, st, b32, (const double *)bp, n);
            if (pre)
                MSB_TRY(pcg_solve<float>(p, w, st, b32, x32, w->v32[2], w->v32[3], w->v32[4], w->v32[5], opts->tol,
                                         opts->maxit, gb, nullptr));
            else
                MSB_TRY(cg_solve<float>(p, w, st, b32, x32, w->v32[2], w->v32[3], w->v32[4], opts->tol, opts->maxit,
                                        gb, nullptr));
            hipLaunchKernelGGL((k_cast<float, double>), dim3(grid_for(n)), dim3(kT), 0, st, u, (const float *)x32, n);
        }
        MSB_TRY(fetch_scal(w, st, 1, B));
        for (int c = 0; c < B; ++c) {
            fl[c] = w->h_int[c] == CAPPED ? RUNNING : w->h_int[c];
            inner[c] = w->h_int[B + c];
            outer[c] = 1;
        }
        if (prec == MSB_FP64) {
            // The CG recurrence residual drifts from b' - K u.  A case whose recurrence met
            // tol but whose FP64 residual does not restarts CG on that residual (residual
            // replacement), aiming at half the missing factor, up to kPolish times.
            CallBuf skip_buf;
            MSB_HIP(hipMalloc(&skip_buf.p, sizeof(int) * B));
            int *skip = static_cast<int *>(skip_buf.p);
            double *r64 = w->v64[2], *d64 = tmp;
            std::vector<int> hskip(B, 0);
            std::vector<double> t2(B, 0.0);
            int used = 0;
            for (int c = 0; c < B; ++c) used = std::max(used, inner[c]);
            for (int j = 0; j < kPolish && used < opts->maxit; ++j) {
                MSB_TRY(true_residual(p, w, st, u, bp, r64, 0));
                MSB_TRY(fetch_scal(w, st, 1, B));
                bool any = false;
                for (int c = 0; c < B; ++c) {
                    const double rr = w->h_scal[c];
                    const double relc = bb[c] > 0 ? std::sqrt(rr / bb[c]) : 0.0;
                    hskip[c] = !(fl[c] == CONVERGED && relc > opts->tol);
                    const double ratio = hskip[c] ? 0.5 : std::min(0.5, 0.5 * opts->tol * std::sqrt(bb[c] / rr));
                    t2[c] = ratio * ratio;
                    any = any || !hskip[c];
                }
                if (!any) break;
                double *t2d = w->scal + 15 * (size_t)B;
                MSB_HIP(hipMemcpyAsync(t2d, t2.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
                MSB_HIP(hipMemcpyAsync(skip, hskip.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
                // rhs = r64 is copied into the CG residual vector r64 itself (same index)
                if (pre)
                    MSB_TRY(pcg_solve<double>(p, w, st, r64, d64, r64, w->v64[3], w->v64[4], w->v64[5], opts->tol,
                                              opts->maxit - used, gb, skip, nullptr, t2d));
                else
                    MSB_TRY(cg_solve<double>(p, w, st, r64, d64, r64, w->v64[3], w->v64[4], opts->tol,
                                             opts->maxit - used, gb, skip, nullptr, nullptr, t2d));
                MSB_TRY(fetch_scal(w, st, 0, B));
                int mx = 0;
                for (int c = 0; c < B; ++c) {
                    if (hskip[c]) continue;
                    inner[c] += w->h_int[B + c];
                    outer[c] += 1;
                    const int f = w->h_int[c] == CAPPED ? RUNNING : w->h_int[c];
                    if (f != CONVERGED) fl[c] = f;
                    mx = std::max(mx, w->h_int[B + c]);
                }
                used += mx;
                hipLaunchKernelGGL(k_add_to<double>, dim3(grid_for(n)), dim3(kT), 0, st, u, (const double *)d64, n);
            }
        }
    } else {
        // FP32 inner CG inside FP64 refinement.  Each inner run reduces the FP32
        // residual by inner_tol (default 0.1 with reliable updates, 1e-4 restarted);
        // then u += d in FP64, the residual is replaced by the FP64 true residual
        // r = b' - K u, and (reliable_update) CG continues with its search direction,
        // or restarts from the new residual (plain iterative refinement).
        const bool reliable = opts->reliable_update != 0;
        const double itol = opts->inner_tol > 0 ? opts->inner_tol : (reliable ? 0.1 : 1e-4);
        CallBuf skip_buf, prev_buf;
        MSB_HIP(hipMalloc(&skip_buf.p, sizeof(int) * B));
        int *skip = static_cast<int *>(skip_buf.p);
        float *r32 = w->v32[0], *d32 = w->v32[1], *p32 = w->v32[2];
        double *r64 = w->v64[2];
        if (reliable) MSB_HIP(hipMalloc(&prev_buf.p, sizeof(double) * (size_t)B * partial_slots(p)));
        double *prev = static_cast<double *>(prev_buf.p);   // [B][x tiles] r.r (r.z) partials before the replacement
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n)), dim3(kT), 0, st, u, n, 0.0);
        hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n)), dim3(kT), 0, st, p32, n, 0.0f);
        hipLaunchKernelGGL((k_cast<double, double>), dim3(grid_for(n)), dim3(kT), 0, st, r64, (const double *)bp, n);
        std::vector<double> rr(bb), best(bb);
        std::vector<int> stall(B, 0);
        int used = 0;
        bool first = true;
        std::vector<int> hskip(B, 0);
        for (int j = 0; j < 1000; ++j) {
            bool all = true;
            for (int c = 0; c < B; ++c) {
                rel[c] = bb[c] > 0 ? std::sqrt(rr[c] / bb[c]) : 0.0;
                if (!std::isfinite(rel[c])) fl[c] = NONFINITE;
                if (fl[c] == RUNNING && rel[c] <= opts->tol) fl[c] = CONVERGED;
                hskip[c] = fl[c] != RUNNING;
                all = all && hskip[c];
            }
            if (all || used >= opts->maxit) break;
            // inner target per case: reduce by itol, but not below what the outer
            // tolerance needs for that case
            std::vector<double> t2(B, itol * itol);
            for (int c = 0; c < B; ++c) {
                double ratio = itol;
                if (!hskip[c] && rr[c] > 0) ratio = std::max(ratio, 0.5 * opts->tol * std::sqrt(bb[c] / rr[c]));
                ratio = std::min(ratio, 0.5);
                t2[c] = ratio * ratio;
            }
            double *t2d = w->scal + 15 * (size_t)B;
            MSB_HIP(hipMemcpyAsync(t2d, t2.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
            MSB_HIP(hipMemcpyAsync(skip, hskip.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n)), dim3(kT), 0, st, r32, (const double *)r64, n);
            if (pre)
                MSB_TRY(pcg_solve<float>(p, w, st, r32, d32, p32, w->v32[3], w->v32[4], w->v32[5], itol,
                                         opts->maxit - used, gb, skip, nullptr, t2d,
                                         (reliable && !first) ? prev : nullptr));
            else
                MSB_TRY(cg_solve<float>(p, w, st, r32, d32, p32, w->v32[3], w->v32[4], itol, opts->maxit - used, gb,
                                        skip, (reliable && !first) ? prev : nullptr, nullptr, t2d));
            first = false;
            MSB_TRY(fetch_scal(w, st, 0, B));
            int mx = 0;
            for (int c = 0; c < B; ++c) {
                if (!hskip[c]) {
                    inner[c] += w->h_int[B + c];
                    outer[c] += 1;
                    if (w->h_int[c] == BREAKDOWN || w->h_int[c] == NONFINITE) fl[c] = w->h_int[c];
                }
                mx = std::max(mx, w->h_int[B + c]);
            }
            used += mx;
            if (reliable) {
                // r.r partials [parity] (CG: x tiles of the prologue, or blocks of the fused
                // steps) or the first array of the r.z partials [parity][3][B][tpc] (PCG)
                const PassArgs<float> pa32 = pass_args<float>(p, p->op);
                const int tpc = x_tiles_per_case(p, pa32.F);
                const RrLayout lay = cg_rr_layout(p, pa32);
                if (pre)
                    hipLaunchKernelGGL(k_save_last, dim3(B), dim3(64), 0, st, (const double *)w->part_rz,
                                       3 * (size_t)B * tpc, (const int *)w->iters, tpc, prev);
                else
                    hipLaunchKernelGGL(k_save_last, dim3(B), dim3(64), 0, st, (const double *)w->part_rr, lay.stride,
                                       (const int *)w->iters, lay.per_case, prev);
            }
            hipLaunchKernelGGL(k_add_to<float>, dim3(grid_for(n)), dim3(kT), 0, st, u, (const float *)d32, n);
            MSB_TRY(true_residual(p, w, st, u, bp, r64, 0));
            MSB_TRY(fetch_scal(w, st, 1, B));
            for (int c = 0; c < B; ++c) {
                if (hskip[c]) continue;
                rr[c] = w->h_scal[c];
                // stagnation: three replacements without a 10% gain on the best residual
                if (rr[c] < 0.81 * best[c]) {
                    best[c] = rr[c];
                    stall[c] = 0;
                } else if (++stall[c] >= 3 && fl[c] == RUNNING) {
                    fl[c] = -1;
                }
            }
        }
        for (int c = 0; c < B; ++c)
            if (fl[c] == -1) fl[c] = RUNNING;   // reported as no convergence below
    }

    // certify: FP64 residual of the final u on free DOFs
    MSB_TRY(true_residual(p, w, st, u, bp, tmp, 0));
    if (p->fixed) hipLaunchKernelGGL(k_set_fixed<double>, dim3(grid_for(n)), dim3(kT), 0, st, u, g, (const uint8_t *)p->fixed, n, dn);
    MSB_TRY(fetch_scal(w, st, 1, B));
    MSB_HIP(hipEventRecord(w->ev_out, st));
    MSB_HIP(hipStreamWaitEvent(user, w->ev_out, 0));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int c = 0; c < B; ++c) {
        rel[c] = bb[c] > 0 ? std::sqrt(w->h_scal[c] / bb[c]) : 0.0;
        msb_status s = flag_status(fl[c]);
        if (s == MSB_OK && !(rel[c] <= opts->tol)) s = MSB_ENOCONV;   // certified residual
        if (fl[c] == RUNNING) s = rel[c] <= opts->tol ? MSB_OK : MSB_ENOCONV;
        info[c].status = s;
        info[c].outer_iters = outer[c];
        info[c].inner_iters = inner[c];
        info[c].rel_residual = rel[c];
        info[c].seconds = secs;
        if (s != MSB_OK && result == MSB_OK) {
            result = s;
            set_error("case %d: %s (relative residual %.3e after %d iterations)", c,
                      s == MSB_ENOTSPD ? "CG breakdown: operator not positive definite on the free DOFs"
                                       : "no convergence", rel[c], inner[c]);
        }
    }
    return result;
}

// ---------------------------------------------------------------------------- Verlet
template <typename T>
static msb_status vv_init_t(msb_plan_s *p, const T *u, const T *bf, T *a, hipStream_t st) {
    EndArgs<T> e = end_args<T>();
    e.epi = EPI_APPLY;
    e.out = a;
    MSB_TRY(product<T>(p, p->op, u, e, st));
    const size_t n = (size_t)p->B * p->dim * p->N, dn = (size_t)p->dim * p->N;
    hipLaunchKernelGGL(k_vv_accel<T>, dim3(grid_for(n)), dim3(kT), 0, st, a, bf, (const uint8_t *)p->fixed, n, dn, p->rho);
    MSB_HIP(hipGetLastError());
    return MSB_OK;
}

extern "C" msb_status msb_vv_init(msb_plan p, msb_precision prec, const void *u, const void *b, void *a, void *stream) {
    MSB_TRY(check_plan(p));
    MSB_CHECK(u && b && a && a != u && a != b, MSB_EINVAL, "bad vectors");
    if (prec == MSB_FP64) return vv_init_t<double>(p, (const double *)u, (const double *)b, (double *)a, (hipStream_t)stream);
    MSB_CHECK(prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    return vv_init_t<float>(p, (const float *)u, (const float *)b, (float *)a, (hipStream_t)stream);
}

template <typename T>
static msb_status vv_run_t(msb_plan_s *p, double dt, int64_t nsteps, T *u, T *v, T *a, const T *bf, const T *g,
                           double *energy, int every, hipStream_t st) {
    SolverWs *w = nullptr;
    MSB_TRY(get_ws(p, w));
    const int64_t ne = (energy && every > 0) ? nsteps / every : 0;
    if (ne > 0 && (size_t)ne > w->energy_cap) {
        if (w->energy) (void)hipFree(w->energy);
        MSB_HIP(hipMalloc(&w->energy, sizeof(double) * ne));
        w->energy_cap = ne;
    }
    if (ne > 0) hipLaunchKernelGGL(k_fill_int<int>, dim3(1), dim3(64), 0, st, w->ecount, 1, 0);
    PassArgs<T> pa = pass_args<T>(p, p->op);
    const int tiles = p->B * pa.ept;   // epilogue partials of the whole batch
    double V = 1.0;
    for (int q = 0; q < p->dim; ++q) V *= p->h;
    // The first step's displacement update runs as the prologue (in place); after that each
    // step's epilogue writes the next displacement into the other of two vectors (u and a
    // workspace copy, alternating), so steps 2.. are the product kernels alone.
    T *us[2] = {u, u};
    if (nsteps > 1) {
        T **alt = alt_vectors<T>(w);
        if (!alt[0]) MSB_HIP(hipMalloc(&alt[0], sizeof(T) * w->nvec));
        us[1] = alt[0];
    }
    for (int64_t s = 1; s <= nsteps; ++s) {
        T *uc = us[(s - 1) & 1];   // u of this step (after its update)
        EndArgs<T> e = end_args<T>();
        e.pro = s == 1 ? PRO_VV_U : PRO_NONE;
        e.pio = uc;
        e.pr = v;
        e.pa = a;
        e.pg = g;
        e.dt = dt;
        e.epi = EPI_VV;
        e.uin = uc;
        e.rhs = bf;
        e.ev = v;
        e.ea = a;
        e.u_next = s < nsteps ? us[s & 1] : nullptr;
        e.rho = p->rho;
        const bool en = ne > 0 && (s % every) == 0 && s / every <= ne;
        e.energy = en ? 1 : 0;
        e.part = en ? w->part_x : nullptr;
        MSB_TRY(launch_product<T>(pa, e, st));
        if (en) hipLaunchKernelGGL(k_energy, dim3(1), dim3(kT), 0, st, (const double *)w->part_x, tiles, p->rho, V, w->energy, w->ecount);
    }
    if (nsteps > 1 && ((nsteps - 1) & 1))   // the last step's u is the workspace copy
        MSB_HIP(hipMemcpyAsync(u, us[1], sizeof(T) * w->nvec, hipMemcpyDeviceToDevice, st));
    MSB_HIP(hipGetLastError());
    if (ne > 0) {
        MSB_HIP(hipMemcpyAsync(energy, w->energy, sizeof(double) * ne, hipMemcpyDeviceToHost, st));
        MSB_HIP(hipStreamSynchronize(st));
    }
    return MSB_OK;
}

// ---------------------------------------------------------------------------- relaxation
// Dynamic relaxation (Alg. 1, CDEI, time step 1): each step is one product chain whose
// x-forward applies the velocity and displacement update with the damping of the
// previous force evaluation, and whose x-inverse forms F = A u + b and the damping
// partials u.K1.u and u.u.
template <typename T>
static msb_status adr_run_t(msb_plan_s *p, msb_precision prec, int64_t nsteps, int restart, T *u, T *v, T *F,
                            const T *bf, const T *g, double *res, hipStream_t st) {
    SolverWs *w = nullptr;
    MSB_TRY(get_ws(p, w));
    const int B = p->B;
    const size_t n = w->nvec, dn = (size_t)p->dim * p->N;
    if (!restart)
        MSB_CHECK(w->adr_prec == (int)prec, MSB_EINVAL,
                  "continuing a relaxation needs an earlier msb_adr_run on this plan in the same precision");
    if (restart || w->adr_version != p->op_version) {   // D for the current operator
        std::vector<double> D;
        int slots = 0;
        build_adr_density(p, D, slots);
        if (w->adr_D64) (void)hipFree(w->adr_D64);
        if (w->adr_D32) (void)hipFree(w->adr_D32);
        w->adr_D64 = nullptr;
        w->adr_D32 = nullptr;
        w->adr_prec = -1;          // no continuation unless this rebuild completes
        w->adr_version = -1;
        MSB_HIP(hipMalloc(&w->adr_D64, sizeof(double) * D.size()));
        MSB_HIP(hipMalloc(&w->adr_D32, sizeof(float) * D.size()));
        std::vector<float> D32(D.begin(), D.end());
        MSB_HIP(hipMemcpy(w->adr_D64, D.data(), sizeof(double) * D.size(), hipMemcpyHostToDevice));
        MSB_HIP(hipMemcpy(w->adr_D32, D32.data(), sizeof(float) * D32.size(), hipMemcpyHostToDevice));
        w->adr_slots = slots;
        w->adr_version = p->op_version;
        if (!w->part_adr) MSB_HIP(hipMalloc(&w->part_adr, sizeof(double) * 3 * (size_t)B * partial_slots(p)));
    }
    const T *D = sizeof(T) == 8 ? (const T *)(const void *)w->adr_D64 : (const T *)(const void *)w->adr_D32;
    const size_t dstride = w->adr_slots > 1 ? dn : 0;
    PassArgs<T> pa = pass_args<T>(p, p->op);
    const int tpc = pa.ept;   // damping partials per case (written by the product's epilogue)
    MSB_CHECK(restart || w->adr_tiles == tpc, MSB_EINVAL,
              "continuing a relaxation needs the launch configuration of the run it continues");
    const size_t nt = (size_t)B * tpc;
    if (restart) {
        if (p->fixed)
            hipLaunchKernelGGL(k_set_fixed<T>, dim3(grid_for(n)), dim3(kT), 0, st, u, g, (const uint8_t *)p->fixed, n, dn);
        EndArgs<T> e = end_args<T>();
        e.pio = u;
        e.epi = EPI_ADR;
        e.uin = u;
        e.rhs = bf;
        e.out = F;
        e.pa = D;
        e.pa_stride = dstride;
        MSB_TRY(launch_product<T>(pa, e, st));
    }
    const bool first_pending = restart || w->adr_pending;
    for (int64_t k = 1; k <= nsteps; ++k) {
        const bool first = first_pending && k == 1;
        EndArgs<T> e = end_args<T>();
        e.pro = PRO_ADR_U;
        e.first = first;
        e.pio = u;
        e.cx = v;
        e.cq = F;
        e.pa = D;
        e.pa_stride = dstride;
        e.pg = g;
        e.cg3 = w->part_adr;
        e.n_cg3 = tpc;
        e.s_cg3 = nt;
        if (!first && tpc > kFusedReduceMaxTiles) {
            const SumSrc src{{w->part_adr, w->part_adr + nt, nullptr, nullptr, nullptr}, {tpc, tpc, 0, 0, 0}};
            hipLaunchKernelGGL(k_cg_sums<2>, dim3(B), dim3(kSumT), 0, st, src, w->case4);
            e.case4 = w->case4;
        }
        e.epi = EPI_ADR;
        e.uin = u;
        e.rhs = bf;
        e.ev = v;
        e.out = F;
        e.part = w->part_adr;
        MSB_TRY(launch_product<T>(pa, e, st));
    }
    MSB_HIP(hipGetLastError());
    w->adr_prec = (int)prec;
    w->adr_tiles = tpc;
    w->adr_pending = first_pending && nsteps == 0;
    if (res) {
        hipLaunchKernelGGL(k_dot_parts<T>, dim3(B * w->P), dim3(kT), 0, st, (const T *)F, (const T *)F, w->part_aux,
                           dn, w->P);
        hipLaunchKernelGGL(k_case_sums, dim3(B), dim3(kT), 0, st, (const double *)w->part_aux, w->P, (size_t)w->P,
                           w->scal, 1.0);
        MSB_HIP(hipGetLastError());
        MSB_TRY(fetch_scal(w, st, 1, B));
        for (int b = 0; b < B; ++b) res[b] = std::sqrt(w->h_scal[b]);
    }
    return MSB_OK;
}

extern "C" msb_status msb_adr_run(msb_plan p, msb_precision prec, int64_t nsteps, int restart, void *u, void *v,
                                  void *F, const void *b, const void *g, double *res, void *stream) {
    MSB_TRY(check_plan(p));
    MSB_CHECK(u && v && F && b, MSB_EINVAL, "null vector");
    MSB_CHECK(nsteps >= 0, MSB_EINVAL, "negative step count");
    MSB_CHECK(u != v && u != F && v != F && b != u && b != v && b != F, MSB_EINVAL, "vectors must not overlap");
    hipStream_t st = (hipStream_t)stream;
    if (prec == MSB_FP64)
        return adr_run_t<double>(p, prec, nsteps, restart, (double *)u, (double *)v, (double *)F, (const double *)b,
                                 (const double *)g, res, st);
    MSB_CHECK(prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    return adr_run_t<float>(p, prec, nsteps, restart, (float *)u, (float *)v, (float *)F, (const float *)b,
                            (const float *)g, res, st);
}

extern "C" msb_status msb_vv_run(msb_plan p, msb_precision prec, double dt, int64_t nsteps, void *u, void *v,
                                 void *a, const void *b, const void *g, double *energy, int every, void *stream) {
    MSB_TRY(check_plan(p));
    MSB_CHECK(u && v && a && b, MSB_EINVAL, "null vector");
    MSB_CHECK(std::isfinite(dt) && dt > 0 && nsteps >= 0, MSB_EINVAL, "need dt > 0 and nsteps >= 0");
    MSB_CHECK(!energy || every > 0, MSB_EINVAL, "energy output needs every > 0");
    hipStream_t st = (hipStream_t)stream;
    if (prec == MSB_FP64)
        return vv_run_t<double>(p, dt, nsteps, (double *)u, (double *)v, (double *)a, (const double *)b,
                                (const double *)g, energy, every, st);
    MSB_CHECK(prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    return vv_run_t<float>(p, dt, nsteps, (float *)u, (float *)v, (float *)a, (const float *)b, (const float *)g,
                           energy, every, st);
}

// ---------------------------------------------------------------------------- gradient
extern "C" msb_status msb_grad_infl(msb_plan p, const double *u, const double *wv, double *dL_da, void *stream) {
    MSB_TRY(check_plan(p));
    MSB_CHECK(u && wv && dL_da, MSB_EINVAL, "null argument");
    MSB_CHECK(p->n_infl > 0, MSB_EINVAL, "plan has no influence coefficients");
    SolverWs *w = nullptr;
    MSB_TRY(get_ws(p, w));
    hipStream_t st = (hipStream_t)stream;
    const int B = p->B, K = p->n_infl;
    for (int k = 0; k < K; ++k) {
        MSB_TRY(ensure_dop(p, k));
        const int tpc = pass_args<double>(p, p->dop[k]).ept;   // epilogue partials per case
        // dL/da_k = w . (A_k u)_F
        EndArgs<double> e = end_args<double>();
        e.epi = EPI_DOT;
        e.rhs = wv;
        e.part = w->part_x;
        MSB_TRY(product<double>(p, p->dop[k], u, e, st));
        hipLaunchKernelGGL(k_case_sums, dim3(B), dim3(kT), 0, st, (const double *)w->part_x, tpc, (size_t)tpc,
                           w->scal + (size_t)k * B, 1.0);
    }
    MSB_HIP(hipGetLastError());
    MSB_HIP(hipMemcpyAsync(w->h_scal, w->scal, sizeof(double) * K * B, hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < K; ++k) dL_da[(size_t)b * K + k] = w->h_scal[(size_t)k * B + b];
    return MSB_OK;
}

// ---------------------------------------------------------------------------- gradient without allocation
// The same gradient for callers that cannot allocate device memory: the epilogue partials
// and the per-case sums live in `scratch`, a fixed device array the library holds on every
// GPU it runs on until the process ends, instead of the plan's solver workspace.  Host code
// never passes the array's name to a kernel (in host code it is a stand-in, not a device
// address): the device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that pointer is used.
constexpr size_t kScratchDoubles = (size_t)1 << 20;   // 8 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::vector<double *> g_scratch_ptr;   // per device: scratch's device address (null: not taken yet)

msb_status scratch_for_device(int dev, double **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        MSB_HIP(hipGetDevice(&cur));
        MSB_CHECK(cur == dev, MSB_EDEVICE, "plan's device %d is not the current device %d", dev, cur);
        void *ptr = nullptr;
        const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        MSB_CHECK(err == hipSuccess && ptr, MSB_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(err));
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MSB_OK;
}
}  // namespace

extern "C" msb_status msb_grad_infl_noalloc(msb_plan p, const double *u, const double *wv, double *dL_da,
                                            void *stream) {
    MSB_TRY(check_plan(p));
    MSB_CHECK(u && wv && dL_da, MSB_EINVAL, "null argument");
    MSB_CHECK(p->n_infl > 0, MSB_EINVAL, "plan has no influence coefficients");
    const int B = p->B, K = p->n_infl;
    for (int k = 0; k < K; ++k)
        MSB_CHECK((int)p->dop.size() > k && p->dop[k].count > 0, MSB_EINVAL,
                  "derivative operator %d not built: call msb_grad_infl or msb_apply_dinfl once first", k);
    // partials [3][B * tpc] of the widest operator's launch, then the sums [K][B]
    size_t need = (size_t)K * B;
    int tpc_max = 0;
    for (int k = 0; k < K; ++k) tpc_max = std::max(tpc_max, pass_args<double>(p, p->dop[k]).ept);
    const size_t part_n = 3 * (size_t)B * tpc_max;
    need += part_n;
    MSB_CHECK(need <= kScratchDoubles, MSB_EINVAL,
              "gradient needs %zu doubles of scratch (batch %d x %d partials per case, %d coefficients); the "
              "fixed scratch holds %zu", need, B, tpc_max, K, kScratchDoubles);
    double *scr = nullptr;
    MSB_TRY(scratch_for_device(p->device, &scr));
    double *part = scr, *sums = scr + part_n;
    hipStream_t st = (hipStream_t)stream;
    // every tile of a launch writes its partials, and every case sum is written before it
    // is read: nothing in the scratch needs to start at zero
    for (int k = 0; k < K; ++k) {
        const int tpc = pass_args<double>(p, p->dop[k]).ept;
        EndArgs<double> e = end_args<double>();
        e.epi = EPI_DOT;
        e.rhs = wv;
        e.part = part;
        MSB_TRY(product<double>(p, p->dop[k], u, e, st));
        hipLaunchKernelGGL(k_case_sums, dim3(B), dim3(kT), 0, st, (const double *)part, tpc, (size_t)tpc,
                           sums + (size_t)k * B, 1.0);
    }
    MSB_HIP(hipGetLastError());
    // sums [K][B] -> dL_da [B][K] (host), one strided copy per coefficient
    for (int k = 0; k < K; ++k)
        MSB_HIP(hipMemcpy2DAsync(dL_da + k, sizeof(double) * K, sums + (size_t)k * B, sizeof(double), sizeof(double),
                                 B, hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    return MSB_OK;
}

// ---------------------------------------------------------------------------- plan groups
// Several plans (grids of different sizes, each with its own cases) whose products run
// as one launch per pass: the grid of every kernel covers the tiles of all members, and
// each block takes its member's arguments from device arrays.  The group CG keeps its
// per-case state (flags, counts, thresholds, tile partials) in contiguous arrays over
// all members' cases, so one host check covers the whole group.
struct msb_group_s {
    std::vector<msb_plan_s *> m;
    int dim = 2, n = 0, Btot = 0, device = 0;
    std::vector<int> case_off;                 // [n + 1]
    msb_launch_config cfg[2];                  // common launch configuration per precision
    std::vector<int> start[2][4];              // host workgroup offsets per pass [n + 1]: x, line, 3D y, tiled
    size_t lds[2][4] = {};
    bool composite[2] = {};
    bool tiled[2] = {};                        // 2D tiled product (tile > 0) in this precision
    std::vector<int> ept[2];                   // epilogue partial sums per case of each member [n]
    std::vector<size_t> poff;                  // member offsets into the partial arrays [n + 1]
    int *dstart[2] = {};                       // device copies [4][n + 1]
    void *dA[2] = {};                          // device PassArgs<T>[n]
    void *dAp[2] = {};                         // device PassArgs<T>[n] of the preconditioners
    void *dE[2] = {};                          // device EndArgs<T>[kSlots][n]
    double *part_x = nullptr, *part_rr = nullptr;   // [3][tiles], [2][tiles] (largest precision)
    double *part_rz = nullptr;                      // [2][3][tiles]: r.z partials by iteration parity
    size_t tiles_max = 0;                           // partial slots of every member (poff[n])
    double *thresh = nullptr, *scal = nullptr;      // [Btot], [16][Btot]
    int *done = nullptr, *iters = nullptr, *skip = nullptr;   // [Btot]
    double *h_scal = nullptr;                  // pinned [16][Btot]
    int *h_int = nullptr;                      // pinned [2][Btot]
    std::vector<int64_t> layout_seen;          // members' layout versions the tile tables were built for
    hipStream_t st = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // captured iteration blocks kept across group CG runs: one per work list seen (members
    // leave the list as they converge), replaced oldest first
    static constexpr int kGraphs = 32;
    SolverWs::CgGraph graphs[kGraphs];
    int graph_next = 0;
    double *case4 = nullptr;                   // [Btot][5] per-case CG sums (members with many tiles)
    bool cg_fused = false;                     // the running group CG fuses its steps into the tiled kernel
    void *dS = nullptr;                        // device GroupSum[kSlots][n]: their sources per slot
    int *dcase = nullptr;                      // [n + 1] case offsets of the members a launch covers
};

namespace msb {
namespace {

// argument slots of a group: CG iterations (first; even and odd partial-sum parity;
// the final update-only iteration of each parity; with the preconditioner these are
// the slots of the preconditioner chain and G_PA_* those of the stiffness chain) and
// one-off products
enum GroupSlot {
    G_FIRST, G_EVEN, G_ODD, G_UPD_EVEN, G_UPD_ODD, G_PA_FIRST, G_PA_EVEN, G_PA_ODD, G_LIFT, G_RESID, G_CERT, kSlots
};

msb_status group_geometry(msb_group_s *g, int f) {
    const bool f32 = f == 1;
    for (int k = 0; k < 4; ++k) g->start[f][k].assign(g->n + 1, 0);
    g->composite[f] = false;
    g->tiled[f] = g->dim == 2 && g->cfg[f].tile > 0;
    g->ept[f].assign(g->n, 0);
    for (int k = 0; k < 4; ++k) g->lds[f][k] = 0;
    for (int i = 0; i < g->n; ++i) {
        int t[4];
        size_t l[4];
        pass_tiles(g->m[i], g->cfg[f], f32, t, l);
        for (int k = 0; k < 4; ++k) {
            g->start[f][k][i + 1] = g->start[f][k][i] + g->m[i]->B * t[k];
            g->lds[f][k] = std::max(g->lds[f][k], l[k]);
        }
        g->ept[f][i] = g->tiled[f] ? t[3] : t[0];
        g->composite[f] = g->composite[f] || plan_needs_composite(g->m[i], f32, g->cfg[f].max_radix);
    }
    std::vector<int> h;
    for (int k = 0; k < 4; ++k) h.insert(h.end(), g->start[f][k].begin(), g->start[f][k].end());
    MSB_HIP(hipMemcpy(g->dstart[f], h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice));
    return MSB_OK;
}

// common configuration: the largest member's, if every member accepts it, else a
// conservative one (one row / one line per workgroup, whole-workgroup teams, no tiles).
// Tiled group products take one block per workgroup (tile_run 1): a run of blocks would
// cross the members' boundaries.
msb_status group_config(msb_group_s *g, int f, const msb_launch_config *want) {
    const bool f32 = f == 1;
    msb_launch_config c;
    if (want) {
        MSB_CHECK(want->tile == 0 || want->tile_run == 1, MSB_EINVAL,
                  "tiled plan-group products take one block per workgroup (tile_run must be 1, got %d)",
                  want->tile_run);
        c = *want;
    } else {
        int big = 0;
        for (int i = 1; i < g->n; ++i)
            if (g->m[i]->N * g->m[i]->B > g->m[big]->N * g->m[big]->B) big = i;
        c = g->m[big]->cfg[f];
        c.tile_run = 1;
    }
    bool ok = true;
    for (int i = 0; i < g->n && ok; ++i) ok = check_config(g->m[i], f32, c) == MSB_OK;
    if (!ok && !want) {
        c = msb_launch_config{1, 0, 1, 1, 256, 1, 0, 1, 256, 8, 0, 0, 256, 0, 1};
        ok = true;
        for (int i = 0; i < g->n && ok; ++i) ok = check_config(g->m[i], f32, c) == MSB_OK;
    }
    MSB_CHECK(ok, want ? MSB_EINVAL : MSB_EUNSUPPORTED, "launch configuration not valid for every member: %s",
              msb_last_error());
    // frame spectra of the members' operators for the tile length
    for (int i = 0; i < g->n && c.tile > 0; ++i) MSB_TRY(ensure_tiles(g->m[i], c.tile, true));
    g->cfg[f] = c;
    return group_geometry(g, f);
}

template <typename T> constexpr int prec_index() { return sizeof(T) == 4 ? 1 : 0; }

// A member's padded lengths may change after the group was built (msb_plan_set_lengths,
// msb_plan_autotune with lengths): its tile counts and LDS sizes change with them.
// Rebuild the tile tables for the current layouts before any group launch; a
// configuration a member no longer accepts falls back to the default group choice.
msb_status group_refresh(msb_group_s *g) {
    bool stale = (int)g->layout_seen.size() != g->n;
    for (int i = 0; i < g->n && !stale; ++i) stale = g->layout_seen[i] != g->m[i]->layout_version;
    if (!stale) return MSB_OK;
    MSB_HIP(hipDeviceSynchronize());
    for (int f = 0; f < 2; ++f) {
        const msb_launch_config keep = g->cfg[f];
        if (group_config(g, f, &keep) != MSB_OK) MSB_TRY(group_config(g, f, nullptr));
    }
    g->layout_seen.resize(g->n);
    for (int i = 0; i < g->n; ++i) g->layout_seen[i] = g->m[i]->layout_version;
    return MSB_OK;
}

// Upload the members' pass arguments (refreshed: operators, constraints and bonds may
// have changed since the last call) and the given end arguments into one slot.
template <typename T> msb_status group_upload_args(msb_group_s *g, std::vector<PassArgs<T>> &A) {
    const int f = prec_index<T>();
    A.resize(g->n);
    for (int i = 0; i < g->n; ++i) {
        // new coefficients drop a member's frame spectra: rebuild those of the group's tile length
        if (g->tiled[f]) MSB_TRY(ensure_tiles(g->m[i], g->cfg[f].tile, true));
        A[i] = pass_args<T>(g->m[i], g->m[i]->op, &g->cfg[f]);
        MSB_CHECK(A[i].tl == (g->tiled[f] ? g->cfg[f].tile : 0), MSB_EDEVICE, "member %d: frame spectra missing", i);
    }
    MSB_HIP(hipMemcpy(g->dA[f], A.data(), sizeof(PassArgs<T>) * g->n, hipMemcpyHostToDevice));
    return MSB_OK;
}
template <typename T> msb_status group_upload_end(msb_group_s *g, int slot, const std::vector<EndArgs<T>> &E) {
    const int f = prec_index<T>();
    EndArgs<T> *dst = static_cast<EndArgs<T> *>(g->dE[f]) + (size_t)slot * g->n;
    MSB_HIP(hipMemcpy(dst, E.data(), sizeof(EndArgs<T>) * g->n, hipMemcpyHostToDevice));
    return MSB_OK;
}
// The members a launch covers: n of them, tile totals per pass; their arguments and
// tile tables are what the device arrays currently hold (all members, or the active
// ones during a group CG).
struct GroupView {
    int n = 0;
    int total[4] = {0, 0, 0, 0};
    int cases = 0;   // cases of the members covered
};

template <typename T> GroupView full_view(const msb_group_s *g) {
    const int f = prec_index<T>();
    GroupView v;
    v.n = g->n;
    for (int k = 0; k < 4; ++k) v.total[k] = g->start[f][k][g->n];
    v.cases = g->Btot;
    return v;
}

template <typename T>
msb_status group_launch(msb_group_s *g, const std::vector<PassArgs<T>> &A, int slot, hipStream_t st,
                        const GroupView *view = nullptr, bool pre = false) {
    const int f = prec_index<T>();
    const GroupView v = view ? *view : full_view<T>(g);
    GroupGrid gg;
    gg.n = v.n;
    gg.start_x = g->dstart[f];
    gg.start_l = g->dstart[f] + (v.n + 1);
    gg.start_y = g->dstart[f] + 2 * (v.n + 1);
    gg.total_x = v.total[0];
    gg.total_l = v.total[1];
    gg.total_y = v.total[2];
    gg.lds_x = g->lds[f][0];
    gg.lds_l = g->lds[f][1];
    gg.lds_y = g->lds[f][2];
    // the preconditioners' chains carry no corrections and stay untiled; the CG slots'
    // end arguments hold a prologue (run first as the transform-free x pass)
    if (g->tiled[f] && !pre) {
        gg.tiled = 1;
        gg.cgq = slot < G_LIFT;
        // fused CG steps carry their update in the tiled kernel: a prologue pass only for the
        // first step (or for every step when not fused)
        gg.pro = slot < G_LIFT && (!g->cg_fused || slot == G_FIRST);
        gg.start_t = g->dstart[f] + 3 * (v.n + 1);
        gg.total_t = v.total[3];
        gg.lds_t = g->lds[f][3];
    }
    const EndArgs<T> *dE = static_cast<const EndArgs<T> *>(g->dE[f]) + (size_t)slot * g->n;
    return launch_group<T>(A[0], gg, static_cast<const PassArgs<T> *>(pre ? g->dAp[f] : g->dA[f]), dE,
                           g->composite[f], st);
}

// Load the device arrays with the members in `act` (argument arrays, the CG slots'
// end arguments and the tile tables); returns the matching view.
template <typename T>
msb_status group_load_members(msb_group_s *g, const std::vector<int> &act, const std::vector<PassArgs<T>> &A,
                              const std::vector<std::vector<EndArgs<T>>> &Eslots, GroupView &v,
                              const std::vector<PassArgs<T>> *Ap = nullptr,
                              const std::vector<std::vector<GroupSum>> *Sslots = nullptr) {
    const int f = prec_index<T>();
    const int na = (int)act.size();
    std::vector<PassArgs<T>> Aa(na), Apa(Ap ? na : 0);
    std::vector<int> st3(4 * (na + 1), 0);
    v.n = na;
    for (int k = 0; k < 4; ++k) v.total[k] = 0;
    for (int j = 0; j < na; ++j) {
        const int i = act[j];
        Aa[j] = A[i];
        if (Ap) Apa[j] = (*Ap)[i];
        for (int k = 0; k < 4; ++k) {
            st3[k * (na + 1) + j + 1] = st3[k * (na + 1) + j] + (g->start[f][k][i + 1] - g->start[f][k][i]);
        }
    }
    for (int k = 0; k < 4; ++k) v.total[k] = st3[k * (na + 1) + na];
    MSB_HIP(hipMemcpy(g->dA[f], Aa.data(), sizeof(PassArgs<T>) * na, hipMemcpyHostToDevice));
    if (Ap) MSB_HIP(hipMemcpy(g->dAp[f], Apa.data(), sizeof(PassArgs<T>) * na, hipMemcpyHostToDevice));
    MSB_HIP(hipMemcpy(g->dstart[f], st3.data(), sizeof(int) * st3.size(), hipMemcpyHostToDevice));
    for (size_t slot = 0; slot < Eslots.size(); ++slot) {
        std::vector<EndArgs<T>> Ea(na);
        for (int j = 0; j < na; ++j) Ea[j] = Eslots[slot][act[j]];
        EndArgs<T> *dst = static_cast<EndArgs<T> *>(g->dE[f]) + slot * g->n;
        MSB_HIP(hipMemcpy(dst, Ea.data(), sizeof(EndArgs<T>) * na, hipMemcpyHostToDevice));
    }
    std::vector<int> cs(na + 1, 0);
    for (int j = 0; j < na; ++j) cs[j + 1] = cs[j] + g->m[act[j]]->B;
    v.cases = cs[na];
    MSB_HIP(hipMemcpy(g->dcase, cs.data(), sizeof(int) * (na + 1), hipMemcpyHostToDevice));
    for (size_t slot = 0; Sslots && slot < Sslots->size(); ++slot) {
        if ((*Sslots)[slot].empty()) continue;
        std::vector<GroupSum> Sa(na);
        for (int j = 0; j < na; ++j) Sa[j] = (*Sslots)[slot][act[j]];
        GroupSum *dst = static_cast<GroupSum *>(g->dS) + slot * g->n;
        MSB_HIP(hipMemcpy(dst, Sa.data(), sizeof(GroupSum) * na, hipMemcpyHostToDevice));
    }
    return MSB_OK;
}

// pending kernels of earlier calls may still read the argument arrays
msb_status group_quiesce(msb_group_s *g, hipStream_t user) {
    MSB_HIP(hipStreamSynchronize(user));
    MSB_HIP(hipStreamSynchronize(g->st));
    return MSB_OK;
}

// Group CG on K d_i = rhs_i for every member, x0 = 0 (restart), like cg_solve; with the
// preconditioners' arguments Ap and the vectors z, preconditioned CG like pcg_solve (two
// group launches per iteration: the preconditioner chain, then the stiffness chain).
template <typename T>
msb_status group_cg(msb_group_s *g, const std::vector<PassArgs<T>> &A, const std::vector<const T *> &rhs,
                    const std::vector<T *> &x, const std::vector<T *> &r, const std::vector<T *> &pv,
                    const std::vector<T *> &q, double tol, int maxit, int graph_block, const int *skip,
                    const double *tol2_case = nullptr, const std::vector<PassArgs<T>> *Ap = nullptr,
                    const std::vector<T *> *z = nullptr, const double *prev = nullptr) {
    // prev (reliable update): [poff] the r.r (r.z) partials of the step that formed each
    // member's kept search direction pv; the first beta continues from them
    const int f = prec_index<T>();
    hipStream_t st = g->st;
    const bool pcg = Ap != nullptr;
    if (pcg && !z) return MSB_EINVAL;
    // plain CG on a tiled configuration whose every member can fuse its steps (see
    // cg_fusable): r, p, q alternate between the caller's vectors and workspace copies
    bool fused = !pcg && g->tiled[f];
    for (int i = 0; i < g->n && fused; ++i) fused = cg_fusable(A[i]);
    std::vector<T *> r1(g->n, nullptr), p1(g->n, nullptr), q1(g->n, nullptr);
    std::vector<SolverWs *> ws(g->n);
    for (int i = 0; i < g->n; ++i) {
        msb_plan_s *p = g->m[i];
        SolverWs *w = nullptr;
        MSB_TRY(get_ws(p, w));
        ws[i] = w;
        const size_t nv = w->nvec;
        if (fused) {
            T **alt = alt_vectors<T>(w);
            for (int k = 0; k < 3; ++k)
                if (!alt[k]) MSB_HIP(hipMalloc(&alt[k], sizeof(T) * nv));
            r1[i] = alt[0], p1[i] = alt[1], q1[i] = alt[2];
        }
        hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(nv)), dim3(kT), 0, st, x[i], nv, T(0));
        if (!prev) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(nv)), dim3(kT), 0, st, pv[i], nv, T(0));
        hipLaunchKernelGGL((k_cast<T, T>), dim3(grid_for(nv)), dim3(kT), 0, st, r[i], rhs[i], nv);
        hipLaunchKernelGGL(k_dot_parts<T>, dim3(p->B * w->P), dim3(kT), 0, st, (const T *)r[i], (const T *)r[i],
                           w->part_aux, (size_t)p->dim * p->N, w->P);
        const int co = g->case_off[i];
        hipLaunchKernelGGL(k_cg_setup, dim3((p->B + 63) / 64), dim3(64), 0, st, (const double *)w->part_aux, w->P,
                           tol * tol, tol2_case ? tol2_case + co : nullptr, g->thresh + co, g->done + co, (size_t)g->Btot,
                           skip ? skip + co : nullptr, g->iters + co, p->B);
    }
    MSB_HIP(hipGetLastError());
    // end arguments of the iteration slots (no kernel of an earlier solve still reads them)
    MSB_HIP(hipStreamSynchronize(st));
    std::vector<std::vector<EndArgs<T>>> Eslots((pcg ? G_PA_ODD : G_UPD_ODD) + 1, std::vector<EndArgs<T>>(g->n));
    // members with many tiles per case take their per-case sums from k_group_sums before the
    // prologue (the rule of the plan alone, so that a member's arithmetic is its own solve's)
    std::vector<std::vector<GroupSum>> Sslots(Eslots.size());
    std::vector<int> many(g->n, 0);
    bool need_sums = false;
    for (int i = 0; i < g->n; ++i) {
        const int tpc = (g->start[f][0][i + 1] - g->start[f][0][i]) / g->m[i]->B;
        many[i] = fused || std::max(tpc, g->ept[f][i]) > kFusedReduceMaxTiles;   // fused steps: always
        need_sums = need_sums || many[i];
    }
    g->cg_fused = fused;
    for (int slot = G_FIRST; slot <= G_UPD_ODD; ++slot) {
        const int parity = (slot == G_ODD || slot == G_UPD_ODD) ? 1 : 0;
        const int prv = (parity + 1) & 1;
        for (int i = 0; i < g->n; ++i) {
            const size_t po = g->poff[i];
            const int nt = g->start[f][0][i + 1] - g->start[f][0][i];
            const int co = g->case_off[i];
            if (fused && slot != G_FIRST) {
                // the whole step in the tiled kernel: previous r, p, q from set prv, new ones to
                // set parity; r.r partials per block at the fused parity stride
                const int B = g->m[i]->B, ept = g->ept[f][i];
                const size_t nrr = (size_t)B * partial_slots(g->m[i]);
                T *rs[2] = {r[i], r1[i]}, *ps[2] = {pv[i], p1[i]}, *qs[2] = {q[i], q1[i]};
                EndArgs<T> e = end_args<T>();
                e.pro = PRO_NONE;
                e.cg_fused = 1;
                e.pio = ps[prv];
                e.cr = rs[prv];
                e.cq = qs[prv];
                e.cx = x[i];
                e.p_new = ps[parity];
                e.r_new = rs[parity];
                e.rr_out = g->part_rr + 2 * po + (size_t)parity * nrr;
                e.update_only = slot == G_UPD_EVEN || slot == G_UPD_ODD;
                e.iters = g->iters + co;
                e.done_prev = g->done + (size_t)prv * g->Btot + co;
                e.done_rw = g->done + (size_t)parity * g->Btot + co;
                e.thresh = g->thresh + co;
                e.epi = EPI_CG_Q;
                e.uin = ps[parity];
                e.out = qs[parity];
                e.rhs = rs[parity];
                e.part = g->part_x + 3 * po;
                const double *rrp = g->part_rr + 2 * po + (size_t)prv * nrr;
                const size_t s3 = (size_t)B * ept;
                GroupSum sm{{rrp, e.part, e.part + s3, e.part + 2 * s3, nullptr}, {ept, ept, ept, ept, 0},
                            g->case4 + 5 * (size_t)co};
                e.case4 = sm.out;
                if (Sslots[slot].empty()) Sslots[slot].resize(g->n);
                Sslots[slot][i] = sm;
                Eslots[slot][i] = e;
                continue;
            }
            EndArgs<T> e = end_args<T>();
            e.pro = pcg ? PRO_PCG_R : PRO_CG_P;
            if (pcg) e.pr = pv[i];
            else e.pio = pv[i];
            e.cx = x[i];
            e.cr = r[i];
            e.cq = q[i];
            e.cg3 = g->part_x + 3 * po;
            e.n_cg3 = g->ept[f][i];
            e.s_cg3 = (size_t)g->m[i]->B * g->ept[f][i];
            e.rr_prev = g->part_rr + 2 * po + (size_t)prv * nt;
            e.rr_out = g->part_rr + 2 * po + (size_t)parity * nt;
            if (fused) {   // the first step: the tile kernel writes the r.r partials per block
                e.rr_out = g->part_rr + 2 * po + (size_t)parity * g->m[i]->B * partial_slots(g->m[i]);
                e.rr_tiles = 1;
            }
            if (pcg) e.rz_k = g->part_rz + (size_t)prv * 3 * g->tiles_max + 3 * po;
            e.first = slot == G_FIRST;
            e.update_only = slot == G_UPD_EVEN || slot == G_UPD_ODD;
            if (slot == G_FIRST && prev && !pcg) {   // continuation: beta = (new r.r) / saved r.r
                e.beta_num = ws[i]->part_aux;
                e.n_num = ws[i]->P;
                e.beta_den = prev + po;
                e.n_den = fused ? g->ept[f][i] : nt / g->m[i]->B;
            }
            e.iters = g->iters + co;
            e.done_prev = g->done + (size_t)prv * g->Btot + co;
            e.case_done = g->done + (size_t)parity * g->Btot + co;
            e.done_rw = g->done + (size_t)parity * g->Btot + co;
            e.thresh = g->thresh + co;
            if (pcg) {   // z = C^-1 r and the partials r.z
                e.epi = EPI_PCG_Z;
                e.uin = r[i];
                e.out = (*z)[i];
                e.sign = 1.0;
                e.part = g->part_rz + (size_t)parity * 3 * g->tiles_max + 3 * po;
            } else {
                e.epi = EPI_CG_Q;
                e.uin = pv[i];
                e.out = q[i];
                e.rhs = r[i];
                e.part = g->part_x + 3 * po;
                e.no_transform = g->tiled[f];   // the tiled product: the x pass is the prologue alone
            }
            GroupSum sm{};
            if (many[i] && slot != G_FIRST) {
                const int tpc = nt / g->m[i]->B, ept = e.n_cg3;
                const double *c3 = e.cg3;
                const size_t s3 = e.s_cg3;
                if (pcg) sm = GroupSum{{e.rr_prev, e.rz_k, c3, c3 + s3, c3 + 2 * s3}, {tpc, tpc, ept, ept, ept}, nullptr};
                else sm = GroupSum{{e.rr_prev, c3, c3 + s3, c3 + 2 * s3, nullptr}, {tpc, ept, ept, ept, 0}, nullptr};
                sm.out = g->case4 + 5 * (size_t)co;
                e.case4 = sm.out;
            }
            if (Sslots[slot].empty()) Sslots[slot].resize(g->n);
            Sslots[slot][i] = sm;
            Eslots[slot][i] = e;
        }
    }
    for (int slot = G_PA_FIRST; pcg && slot <= G_PA_ODD; ++slot) {
        // stiffness chain: p = z + beta p (beta = r.z / previous r.z), q = K p and the
        // partials p.q, r.q, q.q
        const int parity = slot == G_PA_ODD ? 1 : 0;
        const int prv = (parity + 1) & 1;
        for (int i = 0; i < g->n; ++i) {
            const size_t po = g->poff[i];
            EndArgs<T> e = end_args<T>();
            e.pro = PRO_PCG_P;
            e.pr = (*z)[i];
            e.pio = pv[i];
            e.rz_k = g->part_rz + (size_t)parity * 3 * g->tiles_max + 3 * po;
            e.rz_km1 = g->part_rz + (size_t)prv * 3 * g->tiles_max + 3 * po;
            e.first = slot == G_PA_FIRST;
            if (slot == G_PA_FIRST && prev) {   // continuation: beta = (new r.z) / saved r.z
                e.first = false;
                e.rz_km1 = prev + po;
            }
            e.case_done = g->done + (size_t)parity * g->Btot + g->case_off[i];
            e.epi = EPI_CG_Q;
            e.uin = pv[i];
            e.out = q[i];
            e.rhs = r[i];
            e.part = g->part_x + 3 * po;
            e.no_transform = g->tiled[f];
            GroupSum sm{};
            if (many[i] && slot != G_PA_FIRST) {
                const int tpc = (g->start[f][0][i + 1] - g->start[f][0][i]) / g->m[i]->B;
                sm = GroupSum{{e.rz_k, e.rz_km1, nullptr, nullptr, nullptr}, {tpc, tpc, 0, 0, 0},
                              g->case4 + 5 * (size_t)g->case_off[i]};
                e.case4 = sm.out;
            }
            if (Sslots[slot].empty()) Sslots[slot].resize(g->n);
            Sslots[slot][i] = sm;
            Eslots[slot][i] = e;
        }
    }
    // work list: members with a running case (converged or skipped members leave the
    // launches at the next check of the flags, so their tiles cost nothing afterwards)
    std::vector<int> act(g->n);
    for (int i = 0; i < g->n; ++i) act[i] = i;
    GroupView view;
    MSB_TRY(group_load_members<T>(g, act, A, Eslots, view, Ap, &Sslots));
    // A captured block of iterations reads the argument arrays and tile tables at run time;
    // what it fixes is the launch geometry of the view: a graph of an earlier run (the
    // inner solves of the refinement loop) with the same geometry is replayed, not recaptured
    auto graph_key = [&](int block) {
        GraphKey k;
        k.add((int)sizeof(T));
        k.add((int)pcg);
        k.add(A[0]);
        k.add(view.n);
        k.add(view.total);
        k.add(g->lds[f]);
        k.add(g->composite[f]);
        k.add(g->tiled[f]);
        k.add(st);
        k.add(block);
        k.add(view.cases);
        k.add(need_sums);
        k.add(fused);
        return k.b;
    };
    // per-case sums of the members with many tiles, before a slot's prologue (not on the
    // first iteration, whose prologue reduces nothing)
    auto sums = [&](int slot) {
        if (!need_sums || slot == G_FIRST || slot == G_PA_FIRST) return;
        const GroupSum *S = static_cast<const GroupSum *>(g->dS) + (size_t)slot * g->n;
        if (slot >= G_PA_FIRST)
            hipLaunchKernelGGL(k_group_sums<2>, dim3(view.cases), dim3(kSumT), 0, st, S, g->dcase, view.n);
        else if (pcg)
            hipLaunchKernelGGL(k_group_sums<5>, dim3(view.cases), dim3(kSumT), 0, st, S, g->dcase, view.n);
        else
            hipLaunchKernelGGL(k_group_sums<4>, dim3(view.cases), dim3(kSumT), 0, st, S, g->dcase, view.n);
    };
    auto iteration = [&](int it, bool upd) -> msb_status {
        const int slot = upd ? ((it & 1) ? G_UPD_ODD : G_UPD_EVEN) : (it == 0 ? G_FIRST : ((it & 1) ? G_ODD : G_EVEN));
        sums(slot);
        MSB_TRY(group_launch<T>(g, A, slot, st, &view, pcg));
        if (!pcg || upd) return MSB_OK;
        const int slot2 = it == 0 ? G_PA_FIRST : ((it & 1) ? G_PA_ODD : G_PA_EVEN);
        sums(slot2);
        return group_launch<T>(g, A, slot2, st, &view);
    };
    MSB_TRY(iteration(0, false));
    int it = 1;
    const int poll = graph_block > 0 ? graph_block : kPollIterations;
    const int block = poll + (poll & 1);   // even: keeps the partial-sum parity of replays fixed
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    auto find_graph = [&]() -> hipGraphExec_t {
        if (graph_block <= 0) return nullptr;
        const std::vector<unsigned char> k = graph_key(block);
        for (auto &e : g->graphs)
            if (e.exec && e.key == k) return e.exec;
        return nullptr;
    };
    exec = find_graph();
    msb_status s = MSB_OK;
    while (it < maxit && s == MSB_OK) {
        MSB_HIP(hipMemcpyAsync(g->h_int, g->done + (size_t)((it - 1) & 1) * g->Btot, sizeof(int) * g->Btot,
                               hipMemcpyDeviceToHost, st));
        MSB_HIP(hipStreamSynchronize(st));
        std::vector<int> now;
        for (int i = 0; i < g->n; ++i) {
            bool running = false;
            for (int c = g->case_off[i]; c < g->case_off[i + 1]; ++c) running = running || g->h_int[c] == RUNNING;
            if (running) now.push_back(i);
        }
        if (now.empty()) break;
        if (now != act) {   // the stream is idle here (synchronised above)
            act = now;
            MSB_TRY(group_load_members<T>(g, act, A, Eslots, view, Ap, &Sslots));
            exec = find_graph();   // cached graphs stay in the cache
        }
        const int k = std::min(block, maxit - it);
        if (graph_block > 0 && k == block) {
            if (!exec) {
                MSB_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                for (int j = 0; j < block && s == MSB_OK; ++j) s = iteration(it + j, false);
                hipError_t e1 = hipStreamEndCapture(st, &graph);
                if (s != MSB_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    break;
                }
                MSB_HIP(e1);
                hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                if (e2 != hipSuccess) {
                    (void)hipGraphDestroy(graph);
                    MSB_HIP(e2);
                }
                SolverWs::CgGraph &c = g->graphs[g->graph_next];   // kept: replaces the older entry
                g->graph_next = (g->graph_next + 1) % msb_group_s::kGraphs;
                drop_graph(c);
                c.key = graph_key(block);
                c.graph = graph;
                c.exec = exec;
                graph = nullptr;
            }
            MSB_HIP(hipGraphLaunch(exec, st));
        } else {
            for (int j = 0; j < k && s == MSB_OK; ++j) s = iteration(it + j, false);
        }
        it += k;
    }
    if (s == MSB_OK) s = iteration(it, true);   // iteration cap: pending update of running cases
    if (s == MSB_OK && (it & 1))                  // the final flags into slot 0
        MSB_HIP(hipMemcpyAsync(g->done, g->done + g->Btot, sizeof(int) * g->Btot, hipMemcpyDeviceToDevice, st));
    if (s == MSB_OK && fused && (it & 1)) {
        // the last fused step wrote set 1: r, p back for the members it covered (a member that
        // left the work list stopped after an even step, so its vectors are in set 0)
        for (int i : act) {
            MSB_HIP(hipMemcpyAsync(r[i], r1[i], sizeof(T) * ws[i]->nvec, hipMemcpyDeviceToDevice, st));
            MSB_HIP(hipMemcpyAsync(pv[i], p1[i], sizeof(T) * ws[i]->nvec, hipMemcpyDeviceToDevice, st));
        }
    }
    g->cg_fused = false;
    // all members again for the next launches
    MSB_HIP(hipStreamSynchronize(st));
    std::vector<int> all(g->n);
    for (int i = 0; i < g->n; ++i) all[i] = i;
    if (s == MSB_OK) s = group_load_members<T>(g, all, A, Eslots, view, Ap, &Sslots);
    return s;
}

// Reliable updates: each member's r.r (pcg: r.z) partials of the step that formed its search
// direction, into prev + poff[i] (k_save_last), after a group CG run in precision f.
msb_status group_save_last(msb_group_s *g, int f, bool pcg, double *prev, bool fused) {
    for (int i = 0; i < g->n; ++i) {
        const int B = g->m[i]->B;
        const int nt = g->start[f][0][i + 1] - g->start[f][0][i];
        const size_t po = g->poff[i];
        const double *part = pcg ? g->part_rz + 3 * po : g->part_rr + 2 * po;
        // fused steps: r.r partials per block at the parity stride B partial_slots
        const size_t pstride = pcg ? 3 * g->tiles_max : fused ? (size_t)B * partial_slots(g->m[i]) : (size_t)nt;
        const int per = fused && !pcg ? g->ept[f][i] : nt / B;
        hipLaunchKernelGGL(k_save_last, dim3(B), dim3(64), 0, g->st, part, pstride,
                           (const int *)(g->iters + g->case_off[i]), per, prev + po);
    }
    MSB_HIP(hipGetLastError());
    return MSB_OK;
}

// per-case ||rhs_i + A x_i||^2 on free DOFs into g->scal[slot*Btot + case], residual into out_i
msb_status group_residual(msb_group_s *g, const std::vector<PassArgs<double>> &A, int argslot,
                          const std::vector<double *> &x, const std::vector<const double *> &rhs,
                          const std::vector<double *> &out, int slot) {
    std::vector<EndArgs<double>> E(g->n);
    for (int i = 0; i < g->n; ++i) {
        EndArgs<double> e = end_args<double>();
        e.pro = PRO_NONE;
        e.pio = x[i];
        e.uin = x[i];
        e.epi = EPI_RESID;
        e.rhs = rhs[i];
        e.out = out[i];
        e.part = g->part_x + 3 * g->poff[i];
        E[i] = e;
    }
    MSB_TRY(group_quiesce(g, g->st));
    MSB_TRY(group_upload_end<double>(g, argslot, E));
    MSB_TRY(group_launch<double>(g, A, argslot, g->st));
    for (int i = 0; i < g->n; ++i) {
        const int tpc = g->ept[0][i];   // partials per case of the product's epilogue
        hipLaunchKernelGGL(k_case_sums, dim3(g->m[i]->B), dim3(kT), 0, g->st,
                           (const double *)(g->part_x + 3 * g->poff[i]), tpc, (size_t)tpc,
                           g->scal + (size_t)slot * g->Btot + g->case_off[i], 1.0);
    }
    MSB_HIP(hipGetLastError());
    return MSB_OK;
}

msb_status group_fetch(msb_group_s *g, int nslots) {
    MSB_HIP(hipMemcpyAsync(g->h_scal, g->scal, sizeof(double) * nslots * g->Btot, hipMemcpyDeviceToHost, g->st));
    MSB_HIP(hipMemcpyAsync(g->h_int, g->done, sizeof(int) * g->Btot, hipMemcpyDeviceToHost, g->st));
    MSB_HIP(hipMemcpyAsync(g->h_int + g->Btot, g->iters, sizeof(int) * g->Btot, hipMemcpyDeviceToHost, g->st));
    MSB_HIP(hipStreamSynchronize(g->st));
    return MSB_OK;
}

void group_free(msb_group_s *g) {
    for (auto &c : g->graphs) drop_graph(c);
    for (int f = 0; f < 2; ++f) {
        if (g->dstart[f]) (void)hipFree(g->dstart[f]);
        if (g->dA[f]) (void)hipFree(g->dA[f]);
        if (g->dAp[f]) (void)hipFree(g->dAp[f]);
        if (g->dE[f]) (void)hipFree(g->dE[f]);
    }
    void *b[] = {g->part_x, g->part_rr, g->part_rz, g->thresh, g->scal, g->done, g->iters, g->skip, g->case4, g->dS,
                 g->dcase};
    for (void *x : b)
        if (x) (void)hipFree(x);
    if (g->h_scal) (void)hipHostFree(g->h_scal);
    if (g->h_int) (void)hipHostFree(g->h_int);
    if (g->ev_in) (void)hipEventDestroy(g->ev_in);
    if (g->ev_out) (void)hipEventDestroy(g->ev_out);
    if (g->st) (void)hipStreamDestroy(g->st);
    delete g;
}

}  // namespace
}  // namespace msb

extern "C" msb_status msb_group_create(const msb_plan *plans, int nplans, msb_group *out) {
    MSB_CHECK(out, MSB_EINVAL, "null output pointer");
    *out = nullptr;
    MSB_CHECK(plans && nplans >= 1 && nplans <= 4096, MSB_EINVAL, "need 1..4096 plans");
    int dev = -1;
    MSB_HIP(hipGetDevice(&dev));
    for (int i = 0; i < nplans; ++i) {
        MSB_CHECK(plans[i], MSB_EINVAL, "plan %d is null", i);
        MSB_CHECK(plans[i]->dim == plans[0]->dim, MSB_EINVAL, "plan %d: every member must have the same dimension", i);
        MSB_CHECK(plans[i]->device == dev, MSB_EINVAL, "plan %d was created on another device", i);
        for (int j = 0; j < i; ++j) MSB_CHECK(plans[j] != plans[i], MSB_EINVAL, "plan %d is listed twice", i);
    }
    msb_group_s *g = new (std::nothrow) msb_group_s();
    MSB_CHECK(g, MSB_ENOMEM, "host allocation failed");
    g->m.assign(plans, plans + nplans);
    g->n = nplans;
    g->dim = plans[0]->dim;
    g->device = dev;
    g->case_off.assign(nplans + 1, 0);
    for (int i = 0; i < nplans; ++i) g->case_off[i + 1] = g->case_off[i] + plans[i]->B;
    g->Btot = g->case_off[nplans];
    auto fail = [&](msb_status s) {
        group_free(g);
        return s;
    };
    const size_t nb = (size_t)g->Btot;
    for (int f = 0; f < 2; ++f) {
        if (hipMalloc(&g->dstart[f], sizeof(int) * 4 * (nplans + 1)) != hipSuccess) return fail(MSB_ENOMEM);
        const size_t pa = f ? sizeof(PassArgs<float>) : sizeof(PassArgs<double>);
        const size_t ea = f ? sizeof(EndArgs<float>) : sizeof(EndArgs<double>);
        if (hipMalloc(&g->dA[f], pa * nplans) != hipSuccess) return fail(MSB_ENOMEM);
        if (hipMalloc(&g->dAp[f], pa * nplans) != hipSuccess) return fail(MSB_ENOMEM);
        if (hipMalloc(&g->dE[f], ea * kSlots * nplans) != hipSuccess) return fail(MSB_ENOMEM);
        if (f == 0 && (hipMalloc(&g->dS, sizeof(GroupSum) * kSlots * nplans) != hipSuccess ||
                       hipMalloc(&g->dcase, sizeof(int) * (nplans + 1)) != hipSuccess))
            return fail(MSB_ENOMEM);
        msb_status s = group_config(g, f, nullptr);
        if (s != MSB_OK) return fail(s);
    }
    // partial sums sized for any configuration: one x tile per grid row or the blocks of
    // the smallest tiled inner block, whichever is more
    g->poff.assign(nplans + 1, 0);
    for (int i = 0; i < nplans; ++i) g->poff[i + 1] = g->poff[i] + (size_t)plans[i]->B * partial_slots(plans[i]);
    const size_t tiles_max = g->poff[nplans];
    g->tiles_max = tiles_max;
    g->layout_seen.resize(nplans);
    for (int i = 0; i < nplans; ++i) g->layout_seen[i] = plans[i]->layout_version;
    if (hipMalloc(&g->part_x, sizeof(double) * 3 * tiles_max) != hipSuccess ||
        hipMalloc(&g->part_rr, sizeof(double) * 2 * tiles_max) != hipSuccess ||
        hipMalloc(&g->part_rz, sizeof(double) * 6 * tiles_max) != hipSuccess ||
        hipMalloc(&g->thresh, sizeof(double) * nb) != hipSuccess ||
        hipMalloc(&g->case4, sizeof(double) * 5 * nb) != hipSuccess ||
        hipMalloc(&g->scal, sizeof(double) * 16 * nb) != hipSuccess ||
        hipMalloc(&g->done, sizeof(int) * 2 * nb) != hipSuccess || hipMalloc(&g->iters, sizeof(int) * nb) != hipSuccess ||
        hipMalloc(&g->skip, sizeof(int) * nb) != hipSuccess ||
        hipHostMalloc(&g->h_scal, sizeof(double) * 16 * nb) != hipSuccess ||
        hipHostMalloc(&g->h_int, sizeof(int) * 2 * nb) != hipSuccess ||
        hipStreamCreateWithFlags(&g->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming) != hipSuccess) {
        set_error("group allocation failed");
        return fail(MSB_ENOMEM);
    }
    *out = g;
    return MSB_OK;
}

extern "C" msb_status msb_group_set_infl(msb_group g, const double *const *infl, int n_infl, const int *per_case) {
    MSB_CHECK(g, MSB_EINVAL, "null group");
    MSB_CHECK(n_infl == 0 || infl, MSB_EINVAL, "null coefficient array");
    return set_infl_many(g->m.data(), g->n, infl, n_infl, per_case);
}

extern "C" void msb_group_destroy(msb_group g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    group_free(g);
}

extern "C" msb_status msb_group_get_config(msb_group g, msb_precision prec, msb_launch_config *cfg) {
    MSB_CHECK(g && cfg, MSB_EINVAL, "null argument");
    MSB_CHECK(prec == MSB_FP64 || prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    *cfg = g->cfg[prec == MSB_FP32 ? 1 : 0];
    return MSB_OK;
}

extern "C" msb_status msb_group_set_config(msb_group g, msb_precision prec, const msb_launch_config *cfg) {
    MSB_CHECK(g && cfg, MSB_EINVAL, "null argument");
    MSB_CHECK(prec == MSB_FP64 || prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    const int f = prec == MSB_FP32 ? 1 : 0;
    MSB_TRY(group_refresh(g));
    const msb_launch_config keep = g->cfg[f];
    MSB_HIP(hipDeviceSynchronize());
    msb_status s = group_config(g, f, cfg);
    if (s != MSB_OK) {
        g->cfg[f] = keep;
        (void)group_geometry(g, f);
    }
    return s;
}

template <typename T>
static msb_status group_apply_t(msb_group_s *g, const void *const *u, void *const *f, hipStream_t user) {
    for (int i = 0; i < g->n; ++i) {
        MSB_CHECK(u[i] && f[i] && u[i] != f[i], MSB_EINVAL, "member %d: null or aliased vectors", i);
    }
    MSB_TRY(group_quiesce(g, user));
    std::vector<PassArgs<T>> A;
    MSB_TRY(group_upload_args<T>(g, A));
    std::vector<EndArgs<T>> E(g->n);
    for (int i = 0; i < g->n; ++i) {
        EndArgs<T> e = end_args<T>();
        e.pro = PRO_NONE;
        e.pio = (T *)u[i];
        e.uin = (const T *)u[i];
        e.epi = EPI_APPLY;
        e.out = (T *)f[i];
        E[i] = e;
    }
    MSB_TRY(group_upload_end<T>(g, G_LIFT, E));
    return group_launch<T>(g, A, G_LIFT, user);
}

// Group autotuner: the plan autotuner's coordinate search (x passes, line passes, each
// with two-buffer and in-place stages; then the radix cap; then, in 2D, the tiled
// product) over configurations every member accepts, each timed as whole group products
// (HIP events around nrep launches of f_i = A_i u_i on the group's stream).  Leaves the
// fastest in the group.
template <typename T> static msb_status group_tune_t(msb_group_s *g, int effort, double *best_ms) {
    const int f = prec_index<T>();
    const int n = g->n;
    hipStream_t st = g->st;
    std::vector<T *> u(n, nullptr), y(n, nullptr);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Cleanup {
        std::vector<T *> &u, &y;
        hipEvent_t &e0, &e1;
        ~Cleanup() {
            for (T *x : u)
                if (x) (void)hipFree(x);
            for (T *x : y)
                if (x) (void)hipFree(x);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } cleanup{u, y, e0, e1};
    for (int i = 0; i < n; ++i) {
        const size_t nv = (size_t)g->m[i]->B * g->m[i]->dim * g->m[i]->N;
        MSB_HIP(hipMalloc(&u[i], sizeof(T) * nv));
        MSB_HIP(hipMalloc(&y[i], sizeof(T) * nv));
        hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(nv)), dim3(kT), 0, st, u[i], nv, T(1));
    }
    MSB_HIP(hipGetLastError());
    MSB_HIP(hipEventCreate(&e0));
    MSB_HIP(hipEventCreate(&e1));
    int nrep = 3;
    auto time_now = [&](double &ms) -> msb_status {
        std::vector<PassArgs<T>> A;
        MSB_TRY(group_upload_args<T>(g, A));
        std::vector<EndArgs<T>> E(n);
        for (int i = 0; i < n; ++i) {
            EndArgs<T> e = end_args<T>();
            e.pro = PRO_NONE;
            e.pio = u[i];
            e.uin = u[i];
            e.epi = EPI_APPLY;
            e.out = y[i];
            E[i] = e;
        }
        MSB_TRY(group_upload_end<T>(g, G_LIFT, E));
        MSB_TRY(group_launch<T>(g, A, G_LIFT, st));
        MSB_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < nrep; ++r) MSB_TRY(group_launch<T>(g, A, G_LIFT, st));
        MSB_HIP(hipEventRecord(e1, st));
        MSB_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        MSB_HIP(hipEventElapsedTime(&t, e0, e1));
        ms = (double)t / nrep;
        return MSB_OK;
    };
    msb_launch_config best = g->cfg[f];
    best.tile = 0, best.tile_regs = 0, best.tile_run = 1;   // the chain's settings first, the tiled product last
    MSB_TRY(group_config(g, f, &best));
    double bt = 0.0;
    MSB_TRY(time_now(bt));
    nrep = std::max(3, std::min(40, (int)std::ceil(2.0 / std::max(bt, 1e-3))));   // about 2 ms per candidate
    MSB_TRY(time_now(bt));
    msb_status err = MSB_OK;
    auto consider = [&](const msb_launch_config &c) {
        if (err != MSB_OK || group_config(g, f, &c) != MSB_OK) return;   // not valid for every member
        double ms = 0.0;
        err = time_now(ms);
        if (err == MSB_OK && ms < bt) {
            bt = ms;
            best = c;
        }
    };
    const std::vector<int> Fs = {1, 2, 4, 8, 16};
    const std::vector<int> ths = effort ? std::vector<int>{128, 256, 512} : std::vector<int>{256};
    const std::vector<int> sls = effort ? std::vector<int>{1, 2, 4} : std::vector<int>{1, 2};
    const std::vector<int> lps = effort ? std::vector<int>{1, 2, 4} : std::vector<int>{1};
    for (int ip = 0; ip < 2; ++ip)
        for (int F : Fs) {
            for (int th : ths) {
                msb_launch_config c = best;
                c.team_x = 0, c.rows_per_wg = F, c.threads_x = th, c.lds_inplace = (best.lds_inplace & ~1) | ip;
                consider(c);
            }
            for (int sl : sls) {
                msb_launch_config c = best;
                c.team_x = 1, c.rows_per_wg = F, c.slots_fwd = c.slots_inv = sl;
                c.lds_inplace = (best.lds_inplace & ~1) | ip;
                consider(c);
            }
        }
    for (int ip = 0; ip < 2; ++ip)
        for (int Fl : Fs) {
            for (int th : ths) {
                msb_launch_config c = best;
                c.team_line = 0, c.lines_per_wg = Fl, c.threads_line = th;
                c.lds_inplace = (best.lds_inplace & ~2) | (ip << 1);
                consider(c);
            }
            for (int lp : lps) {
                msb_launch_config c = best;
                c.team_line = 1, c.lines_per_wg = Fl, c.lines_per_wave = lp;
                c.lds_inplace = (best.lds_inplace & ~2) | (ip << 1);
                consider(c);
            }
        }
    for (int r : {4, 8, 16}) {
        msb_launch_config c = best;
        c.max_radix = r;
        consider(c);
    }
    if (g->dim == 2) {
        // the tiled product over the members' blocks (one block per workgroup): LDS frames of
        // several lengths, then register-resident frames; the chain's settings stay for the
        // preconditioners and the solver prologues
        const msb_launch_config chain = best;
        const std::vector<int> tls = effort ? std::vector<int>{16, 20, 24, 30, 32, 36, 40, 48, 60, 64}
                                            : std::vector<int>{24, 32, 40, 48, 64};
        for (int tl : tls)
            for (int th : ths) {
                msb_launch_config c = chain;
                c.tile = tl, c.threads_tile = th, c.tile_regs = 0, c.tile_run = 1;
                consider(c);
            }
        for (int tl : {16, 32, 64}) {
            msb_launch_config c = chain;
            c.tile = tl, c.tile_regs = 1, c.tile_run = 1;
            consider(c);
        }
    }
    MSB_TRY(err);
    MSB_TRY(group_config(g, f, &best));
    if (best_ms) *best_ms = bt;
    return MSB_OK;
}

extern "C" msb_status msb_group_autotune(msb_group g, msb_precision prec, int effort, msb_launch_config *best,
                                         double *best_ms) {
    MSB_CHECK(g, MSB_EINVAL, "null group");
    MSB_CHECK(prec == MSB_FP64 || prec == MSB_FP32 || prec == MSB_FP32_REFINED, MSB_EINVAL, "bad precision");
    MSB_CHECK(effort == 0 || effort == 1, MSB_EINVAL, "effort must be 0 or 1");
    int dev = -1;
    MSB_HIP(hipGetDevice(&dev));
    MSB_CHECK(dev == g->device, MSB_EINVAL, "group was created on device %d, current is %d", g->device, dev);
    MSB_TRY(group_refresh(g));
    MSB_HIP(hipDeviceSynchronize());
    double t64 = 0.0, t32 = 0.0;
    if (prec != MSB_FP32) MSB_TRY(group_tune_t<double>(g, effort, &t64));
    if (prec != MSB_FP64) MSB_TRY(group_tune_t<float>(g, effort, &t32));
    if (best) *best = g->cfg[prec == MSB_FP64 ? 0 : 1];
    if (best_ms) *best_ms = prec == MSB_FP64 ? t64 : t32;
    return MSB_OK;
}

extern "C" msb_status msb_group_apply(msb_group g, msb_precision prec, const void *const *u, void *const *f,
                                      void *stream) {
    MSB_CHECK(g && u && f, MSB_EINVAL, "null argument");
    int dev = -1;
    MSB_HIP(hipGetDevice(&dev));
    MSB_CHECK(dev == g->device, MSB_EINVAL, "group was created on device %d, current is %d", g->device, dev);
    MSB_TRY(group_refresh(g));
    if (prec == MSB_FP64) return group_apply_t<double>(g, u, f, (hipStream_t)stream);
    MSB_CHECK(prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    return group_apply_t<float>(g, u, f, (hipStream_t)stream);
}

extern "C" msb_status msb_group_solve_static(msb_group g, msb_precision prec, const double *const *b,
                                             const double *const *gv, double *const *u, const msb_solve_opts *opts,
                                             msb_solve_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    MSB_CHECK(g && b && u && opts && info, MSB_EINVAL, "null argument");
    MSB_CHECK(opts->tol > 0 && opts->tol < 1 && opts->maxit > 0, MSB_EINVAL, "need 0 < tol < 1 and maxit > 0");
    MSB_CHECK(prec == MSB_FP64 || prec == MSB_FP32 || prec == MSB_FP32_REFINED, MSB_EINVAL, "bad precision");
    MSB_CHECK(opts->graph_block >= 0 && opts->graph_block <= 4096, MSB_EINVAL, "graph_block out of range");
    MSB_CHECK(opts->precond == 0 || opts->precond == 1, MSB_EINVAL, "precond must be 0 or 1");
    for (int i = 0; i < g->n; ++i)
        MSB_CHECK(!g->m[i]->nu64, MSB_EUNSUPPORTED, "member %d: the surface-corrected operator is not symmetric", i);
    int dev = -1;
    MSB_HIP(hipGetDevice(&dev));
    MSB_CHECK(dev == g->device, MSB_EINVAL, "group was created on device %d, current is %d", g->device, dev);
    MSB_TRY(group_refresh(g));
    const int n = g->n, Bt = g->Btot;
    for (int i = 0; i < n; ++i)
        MSB_CHECK(b[i] && u[i] && b[i] != u[i] && (!gv || gv[i] != u[i]), MSB_EINVAL,
                  "member %d: null or aliased vectors", i);
    hipStream_t user = (hipStream_t)stream;
    MSB_TRY(group_quiesce(g, user));
    hipStream_t st = g->st;
    std::vector<SolverWs *> w(n);
    for (int i = 0; i < n; ++i) MSB_TRY(get_ws(g->m[i], w[i]));
    std::vector<PassArgs<double>> A64;
    std::vector<PassArgs<float>> A32;
    MSB_TRY(group_upload_args<double>(g, A64));
    if (prec != MSB_FP64) MSB_TRY(group_upload_args<float>(g, A32));
    const int gb = opts->graph_block;
    // circulant preconditioners of the members (built on first use), their chains
    // without the corrections
    const bool pre = opts->precond == 1;
    std::vector<PassArgs<double>> P64;
    std::vector<PassArgs<float>> P32;
    std::vector<double *> z64(n);
    std::vector<float *> z32(n);
    if (pre) {
        MSB_TRY(build_preconditioners(g->m.data(), n));   // the missing ones, host work in parallel
        for (int i = 0; i < n; ++i) {
            msb_plan_s *p = g->m[i];
            MSB_TRY(ensure_pre(p));
            if (prec == MSB_FP64) {
                P64.push_back(pass_args<double>(p, p->pre, &g->cfg[0]));
                P64.back().corr = 0;
            } else {
                P32.push_back(pass_args<float>(p, p->pre, &g->cfg[1]));
                P32.back().corr = 0;
            }
            z64[i] = w[i]->v64[5];
            z32[i] = w[i]->v32[5];
        }
    }
    const std::vector<PassArgs<double>> *ap64 = pre ? &P64 : nullptr;
    const std::vector<PassArgs<float>> *ap32 = pre ? &P32 : nullptr;
    const std::vector<double *> *zz64 = pre ? &z64 : nullptr;
    const std::vector<float *> *zz32 = pre ? &z32 : nullptr;

    // lifted right-hand sides b'_i (per member, as msb_solve_static) and their norms
    std::vector<double *> bp(n), tmp(n);
    for (int i = 0; i < n; ++i) {
        msb_plan_s *p = g->m[i];
        const size_t nv = w[i]->nvec, dn = (size_t)p->dim * p->N;
        bp[i] = w[i]->v64[0];
        tmp[i] = w[i]->v64[1];
        const double *gi = gv ? gv[i] : nullptr;
        if (gi && p->fixed) {
            hipLaunchKernelGGL(k_mask_copy<double>, dim3(grid_for(nv)), dim3(kT), 0, st, tmp[i], gi, (const uint8_t *)p->fixed, nv, dn, 1);
            EndArgs<double> e = end_args<double>();
            e.epi = EPI_RESID;
            e.rhs = b[i];
            e.out = bp[i];
            MSB_TRY(product<double>(p, p->op, tmp[i], e, st));
        } else {
            hipLaunchKernelGGL(k_mask_copy<double>, dim3(grid_for(nv)), dim3(kT), 0, st, bp[i], b[i], (const uint8_t *)p->fixed, nv, dn, 0);
        }
        hipLaunchKernelGGL(k_dot_parts<double>, dim3(p->B * w[i]->P), dim3(kT), 0, st, (const double *)bp[i],
                           (const double *)bp[i], w[i]->part_aux, dn, w[i]->P);
        hipLaunchKernelGGL(k_case_sums, dim3(p->B), dim3(kT), 0, st, (const double *)w[i]->part_aux, w[i]->P,
                           (size_t)w[i]->P, g->scal + g->case_off[i], 1.0);
    }
    MSB_HIP(hipGetLastError());
    MSB_TRY(group_fetch(g, 1));
    std::vector<double> bb(g->h_scal, g->h_scal + Bt);
    for (int c = 0; c < Bt; ++c)
        MSB_CHECK(std::isfinite(bb[c]), MSB_EINVAL, "case %d: right-hand side (or lift) is not finite", c);

    std::vector<int> outer(Bt, 0), inner(Bt, 0), fl(Bt, RUNNING);
    std::vector<double> rel(Bt, 0.0);
    std::vector<const double *> cbp(bp.begin(), bp.end());
    if (prec == MSB_FP64) {
        std::vector<double *> r(n), pv(n), q(n), x(u, u + n);
        for (int i = 0; i < n; ++i) r[i] = w[i]->v64[2], pv[i] = w[i]->v64[3], q[i] = w[i]->v64[4];
        MSB_TRY(group_cg<double>(g, A64, cbp, x, r, pv, q, opts->tol, opts->maxit, gb, nullptr, nullptr, ap64, zz64));
        MSB_TRY(group_fetch(g, 1));
        for (int c = 0; c < Bt; ++c) {
            fl[c] = g->h_int[c] == CAPPED ? RUNNING : g->h_int[c];
            inner[c] = g->h_int[Bt + c];
            outer[c] = 1;
        }
        // residual replacement for cases whose recurrence met tol but whose FP64 residual
        // does not (as msb_solve_static)
        std::vector<const double *> rc(r.begin(), r.end());
        std::vector<int> hskip(Bt, 0);
        std::vector<double> t2(Bt, 0.0);
        int used = 0;
        for (int c = 0; c < Bt; ++c) used = std::max(used, inner[c]);
        for (int j = 0; j < kPolish && used < opts->maxit; ++j) {
            MSB_TRY(group_residual(g, A64, G_RESID, x, cbp, r, 0));
            MSB_TRY(group_fetch(g, 1));
            bool any = false;
            for (int c = 0; c < Bt; ++c) {
                const double rr = g->h_scal[c];
                const double relc = bb[c] > 0 ? std::sqrt(rr / bb[c]) : 0.0;
                hskip[c] = !(fl[c] == CONVERGED && relc > opts->tol);
                const double ratio = hskip[c] ? 0.5 : std::min(0.5, 0.5 * opts->tol * std::sqrt(bb[c] / rr));
                t2[c] = ratio * ratio;
                any = any || !hskip[c];
            }
            if (!any) break;
            double *t2d = g->scal + 15 * (size_t)Bt;
            MSB_HIP(hipMemcpyAsync(t2d, t2.data(), sizeof(double) * Bt, hipMemcpyHostToDevice, st));
            MSB_HIP(hipMemcpyAsync(g->skip, hskip.data(), sizeof(int) * Bt, hipMemcpyHostToDevice, st));
            MSB_TRY(group_cg<double>(g, A64, rc, tmp, r, pv, q, opts->tol, opts->maxit - used, gb, g->skip, t2d, ap64,
                                     zz64));
            MSB_TRY(group_fetch(g, 0));
            int mx = 0;
            for (int c = 0; c < Bt; ++c) {
                if (hskip[c]) continue;
                inner[c] += g->h_int[Bt + c];
                outer[c] += 1;
                const int f = g->h_int[c] == CAPPED ? RUNNING : g->h_int[c];
                if (f != CONVERGED) fl[c] = f;
                mx = std::max(mx, g->h_int[Bt + c]);
            }
            used += mx;
            for (int i = 0; i < n; ++i)
                hipLaunchKernelGGL(k_add_to<double>, dim3(grid_for(w[i]->nvec)), dim3(kT), 0, st, u[i],
                                   (const double *)tmp[i], w[i]->nvec);
        }
    } else if (prec == MSB_FP32) {
        std::vector<const float *> b32(n);
        std::vector<float *> x32(n), r(n), pv(n), q(n);
        for (int i = 0; i < n; ++i) {
            const size_t nv = w[i]->nvec;
            hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(nv)), dim3(kT), 0, st, w[i]->v32[0], (const double *)bp[i], nv);
            b32[i] = w[i]->v32[0];
            x32[i] = w[i]->v32[1], r[i] = w[i]->v32[2], pv[i] = w[i]->v32[3], q[i] = w[i]->v32[4];
        }
        MSB_TRY(group_cg<float>(g, A32, b32, x32, r, pv, q, opts->tol, opts->maxit, gb, nullptr, nullptr, ap32, zz32));
        for (int i = 0; i < n; ++i)
            hipLaunchKernelGGL((k_cast<float, double>), dim3(grid_for(w[i]->nvec)), dim3(kT), 0, st, u[i], (const float *)x32[i], w[i]->nvec);
        MSB_TRY(group_fetch(g, 1));
        for (int c = 0; c < Bt; ++c) {
            fl[c] = g->h_int[c] == CAPPED ? RUNNING : g->h_int[c];
            inner[c] = g->h_int[Bt + c];
            outer[c] = 1;
        }
    } else {
        // iterative refinement, as msb_solve_static: FP32 CG on K d = r to a reduction of
        // inner_tol, u += d in FP64, r = b' - K u with the FP64 product; CG restarts, or
        // (reliable_update) keeps each member's search direction across the replacement
        const bool reliable = opts->reliable_update != 0;
        const double itol = opts->inner_tol > 0 ? opts->inner_tol : (reliable ? 0.1 : 1e-4);
        CallBuf prev_buf;
        if (reliable) MSB_HIP(hipMalloc(&prev_buf.p, sizeof(double) * g->tiles_max));
        double *prev = static_cast<double *>(prev_buf.p);
        bool first = true;
        std::vector<const float *> r32c(n);
        std::vector<float *> r32(n), d32(n), p32(n), q32(n), rr32(n);
        std::vector<double *> r64(n), uu(u, u + n);
        for (int i = 0; i < n; ++i) {
            const size_t nv = w[i]->nvec;
            r32[i] = w[i]->v32[0], d32[i] = w[i]->v32[1], p32[i] = w[i]->v32[2], rr32[i] = w[i]->v32[3], q32[i] = w[i]->v32[4];
            r32c[i] = r32[i];
            r64[i] = w[i]->v64[2];
            hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(nv)), dim3(kT), 0, st, u[i], nv, 0.0);
            hipLaunchKernelGGL((k_cast<double, double>), dim3(grid_for(nv)), dim3(kT), 0, st, r64[i], (const double *)bp[i], nv);
        }
        std::vector<double> rr(bb), best(bb);
        std::vector<int> stall(Bt, 0), hskip(Bt, 0);
        int used = 0;
        for (int j = 0; j < 1000; ++j) {
            bool all = true;
            for (int c = 0; c < Bt; ++c) {
                rel[c] = bb[c] > 0 ? std::sqrt(rr[c] / bb[c]) : 0.0;
                if (!std::isfinite(rel[c])) fl[c] = NONFINITE;
                if (fl[c] == RUNNING && rel[c] <= opts->tol) fl[c] = CONVERGED;
                hskip[c] = fl[c] != RUNNING;
                all = all && hskip[c];
            }
            if (all || used >= opts->maxit) break;
            std::vector<double> t2(Bt, itol * itol);   // per-case inner target, as for one plan
            for (int c = 0; c < Bt; ++c) {
                double ratio = itol;
                if (!hskip[c] && rr[c] > 0) ratio = std::max(ratio, 0.5 * opts->tol * std::sqrt(bb[c] / rr[c]));
                ratio = std::min(ratio, 0.5);
                t2[c] = ratio * ratio;
            }
            double *t2d = g->scal + 15 * (size_t)Bt;
            MSB_HIP(hipMemcpyAsync(t2d, t2.data(), sizeof(double) * Bt, hipMemcpyHostToDevice, st));
            MSB_HIP(hipMemcpyAsync(g->skip, hskip.data(), sizeof(int) * Bt, hipMemcpyHostToDevice, st));
            for (int i = 0; i < n; ++i)
                hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(w[i]->nvec)), dim3(kT), 0, st, r32[i], (const double *)r64[i], w[i]->nvec);
            MSB_TRY(group_cg<float>(g, A32, r32c, d32, rr32, p32, q32, itol, opts->maxit - used, gb, g->skip, t2d, ap32,
                                    zz32, (reliable && !first) ? prev : nullptr));
            first = false;
            if (reliable) {
                bool fz = !pre && g->tiled[1];   // the group CG fused its steps (as group_cg decides)
                for (int i = 0; i < n && fz; ++i) fz = cg_fusable(A32[i]);
                MSB_TRY(group_save_last(g, 1, pre, prev, fz));
            }
            MSB_TRY(group_fetch(g, 0));
            int mx = 0;
            for (int c = 0; c < Bt; ++c) {
                if (!hskip[c]) {
                    inner[c] += g->h_int[Bt + c];
                    outer[c] += 1;
                    if (g->h_int[c] == BREAKDOWN || g->h_int[c] == NONFINITE) fl[c] = g->h_int[c];
                }
                mx = std::max(mx, g->h_int[Bt + c]);
            }
            used += mx;
            for (int i = 0; i < n; ++i)
                hipLaunchKernelGGL(k_add_to<float>, dim3(grid_for(w[i]->nvec)), dim3(kT), 0, st, u[i], (const float *)d32[i], w[i]->nvec);
            MSB_TRY(group_residual(g, A64, G_RESID, uu, cbp, r64, 0));
            MSB_TRY(group_fetch(g, 1));
            for (int c = 0; c < Bt; ++c) {
                if (hskip[c]) continue;
                rr[c] = g->h_scal[c];
                if (rr[c] < 0.81 * best[c]) {
                    best[c] = rr[c];
                    stall[c] = 0;
                } else if (++stall[c] >= 3 && fl[c] == RUNNING) {
                    fl[c] = -1;
                }
            }
        }
        for (int c = 0; c < Bt; ++c)
            if (fl[c] == -1) fl[c] = RUNNING;
    }

    // certify: FP64 residual of the final u on free DOFs; u_C = g
    std::vector<double *> uu(u, u + n);
    MSB_TRY(group_residual(g, A64, G_CERT, uu, cbp, tmp, 0));
    for (int i = 0; i < n; ++i) {
        msb_plan_s *p = g->m[i];
        if (p->fixed)
            hipLaunchKernelGGL(k_set_fixed<double>, dim3(grid_for(w[i]->nvec)), dim3(kT), 0, st, u[i],
                               gv ? gv[i] : nullptr, (const uint8_t *)p->fixed, w[i]->nvec, (size_t)p->dim * p->N);
    }
    MSB_TRY(group_fetch(g, 1));
    MSB_HIP(hipEventRecord(g->ev_out, st));
    MSB_HIP(hipStreamWaitEvent(user, g->ev_out, 0));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    msb_status result = MSB_OK;
    for (int c = 0; c < Bt; ++c) {
        rel[c] = bb[c] > 0 ? std::sqrt(g->h_scal[c] / bb[c]) : 0.0;
        msb_status s = flag_status(fl[c]);
        if (s == MSB_OK && !(rel[c] <= opts->tol)) s = MSB_ENOCONV;   // certified residual
        if (fl[c] == RUNNING) s = rel[c] <= opts->tol ? MSB_OK : MSB_ENOCONV;
        info[c].status = s;
        info[c].outer_iters = outer[c];
        info[c].inner_iters = inner[c];
        info[c].rel_residual = rel[c];
        info[c].seconds = secs;
        if (s != MSB_OK && result == MSB_OK) {
            result = s;
            set_error("case %d of the group: %s (relative residual %.3e after %d iterations)", c,
                      s == MSB_ENOTSPD ? "CG breakdown: operator not positive definite on the free DOFs"
                                       : "no convergence", rel[c], inner[c]);
        }
    }
    return result;
}
