// Launch configurations of the product's kernels and the autotuner that picks them.
//
// The product f = A u is a fixed chain of LDS-staged transform kernels (x-forward,
// one or three line passes, x-inverse).  How the work is cut into workgroups --
// rows or lines per workgroup, whole-workgroup teams or wave-owned signals, signals
// per wave, threads per workgroup -- and the radix cap of the Stockham schedules
// change only the speed.  The tuner times candidates with HIP events between the
// kernels of the chain, so the x passes and the line passes are chosen on their
// own kernel times (coordinate search), then the radix cap and, optionally, the
// padded lengths.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "common.hpp"
#include "passes.hpp"

namespace msb {

// Deterministic input in [-1, 1): an integer hash of the element index.
template <typename T> __global__ void k_tune_fill(T *x, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 0x9E3779B1u + (uint32_t)(i >> 32);
        h ^= h >> 15;
        h *= 0x85EBCA77u;
        h ^= h >> 13;
        x[i] = T((double)(int32_t)h * (1.0 / 2147483648.0));
    }
}

namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();

// Buffers and events of one tuning run for precision T.
template <typename T> struct Bench {
    msb_plan_s *p;
    hipStream_t st;
    T *u = nullptr, *f = nullptr;
    int np = 0, nrep = 3;
    std::vector<hipEvent_t> ev;
    std::vector<double> ms;

    msb_status init(int max_rep) {
        np = n_passes(p->dim);   // the chain; a tiled candidate times one kernel (ms[0])
        const size_t n = (size_t)p->B * p->dim * p->N;
        MSB_HIP(hipMalloc(&u, sizeof(T) * n));
        MSB_HIP(hipMalloc(&f, sizeof(T) * n));
        hipLaunchKernelGGL(k_tune_fill<T>, dim3(1024), dim3(256), 0, st, u, n);
        MSB_HIP(hipGetLastError());
        ev.assign((size_t)(np + 1) * max_rep, nullptr);
        for (auto &e : ev) MSB_HIP(hipEventCreate(&e));
        ms.assign(np, 0.0);
        return MSB_OK;
    }
    ~Bench() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (u) (void)hipFree(u);
        if (f) (void)hipFree(f);
    }

    // Time the chain under configuration c; returns false if c is not valid here.
    // ms[i] = mean duration of kernel i over nrep products (after one warm-up).
    bool run(const msb_launch_config &c, msb_status &err) {
        const bool f32 = sizeof(T) == 4;
        if (check_config(p, f32, c) != MSB_OK) return false;
        const msb_launch_config keep = p->cfg[f32];
        p->cfg[f32] = c;
        err = set_schedules(p, f32, c.max_radix);
        if (err == MSB_OK) err = ensure_tiles(p);
        if (err == MSB_OK) err = time_now();
        if (err != MSB_OK) {
            p->cfg[f32] = keep;
            (void)set_schedules(p, f32, keep.max_radix);
            return false;
        }
        return true;
    }

    msb_status time_now() {
        PassArgs<T> a = pass_args<T>(p, p->op);
        const int npa = n_passes(a);
        EndArgs<T> e;
        memset(&e, 0, sizeof(e));
        e.pro = PRO_NONE;
        e.epi = EPI_APPLY;
        e.sign = 1.0;
        e.rho = 1.0;
        e.pio = u;
        e.uin = u;
        e.out = f;
        MSB_TRY(launch_product<T>(a, e, st));
        for (int r = 0; r < nrep; ++r) MSB_TRY(launch_product<T>(a, e, st, ev.data() + (size_t)r * (np + 1)));
        MSB_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < np; ++i) {
            double acc = 0.0;
            for (int r = 0; r < nrep && i < npa; ++r) {
                float t = 0.f;
                MSB_HIP(hipEventElapsedTime(&t, ev[(size_t)r * (np + 1) + i], ev[(size_t)r * (np + 1) + i + 1]));
                acc += t;
            }
            ms[i] = acc / nrep;
        }
        return MSB_OK;
    }
    double x_time() const { return ms[0] + ms[np - 1]; }
    double line_time() const {
        double t = 0.0;
        for (int i = 1; i < np - 1; ++i) t += ms[i];
        return t;
    }
    double total() const {
        double t = 0.0;
        for (double v : ms) t += v;
        return t;
    }
};

constexpr int kMaxRep = 40;

// Coordinate search for one precision; leaves the best configuration in the plan
// and its product time (ms) in *best_ms.
template <typename T> msb_status tune_precision(msb_plan_s *p, int effort, hipStream_t st, double *best_ms) {
    const bool f32 = sizeof(T) == 4;
    Bench<T> bn;
    bn.p = p;
    bn.st = st;
    MSB_TRY(bn.init(kMaxRep));
    msb_status err = MSB_OK;
    msb_launch_config cur = p->cfg[f32];
    cur.tile = 0;   // the chain's settings are searched on the chain; the tiled product last
    cur.tile_regs = 0;
    cur.tile_run = 1;
    MSB_CHECK(bn.run(cur, err), err != MSB_OK ? err : MSB_EINVAL, "current configuration is not valid");
    // about 2 ms of kernels per candidate, 3..40 products
    bn.nrep = std::max(3, std::min(kMaxRep, (int)std::ceil(2.0 / std::max(bn.total(), 1e-3))));

    const std::vector<int> Fs = {1, 2, 4, 8, 16};
    const std::vector<int> ths = effort ? std::vector<int>{64, 128, 256, 384, 512} : std::vector<int>{128, 256, 512};
    const std::vector<int> sls = effort ? std::vector<int>{1, 2, 3, 4, 6, 8} : std::vector<int>{1, 2, 4};
    const std::vector<int> lpws = effort ? std::vector<int>{1, 2, 3, 4} : std::vector<int>{1, 2};

    // x passes: (team, rows per workgroup) groups; wave teams pick the forward and
    // inverse slot counts separately from their own kernel times.  ip: the x-pass bit of
    // lds_inplace the candidates take.
    auto scan_x = [&](int ip) -> msb_status {
        msb_launch_config best = cur;
        MSB_TRY(bn.run(cur, err) ? MSB_OK : err);
        double bt = bn.x_time();
        const int ipm = (cur.lds_inplace & ~1) | ip;
        for (int F : Fs) {
            for (int th : ths) {
                msb_launch_config c = cur;
                c.team_x = 0;
                c.rows_per_wg = F;
                c.threads_x = th;
                c.lds_inplace = ipm;
                if (bn.run(c, err) && bn.x_time() < bt) {
                    bt = bn.x_time();
                    best = c;
                }
                MSB_TRY(err);
            }
            double tf = kInf, ti = kInf;
            int sf = 1, si = 1;
            for (int sl : sls) {
                msb_launch_config c = cur;
                c.team_x = 1;
                c.rows_per_wg = F;
                c.slots_fwd = c.slots_inv = sl;
                c.lds_inplace = ipm;
                if (bn.run(c, err)) {
                    if (bn.ms[0] < tf) tf = bn.ms[0], sf = sl;
                    if (bn.ms[bn.np - 1] < ti) ti = bn.ms[bn.np - 1], si = sl;
                }
                MSB_TRY(err);
            }
            if (tf + ti < bt) {
                msb_launch_config c = cur;
                c.team_x = 1;
                c.rows_per_wg = F;
                c.slots_fwd = sf;
                c.slots_inv = si;
                c.lds_inplace = ipm;
                if (check_config(p, f32, c) == MSB_OK) {
                    bt = tf + ti;
                    best = c;
                }
            }
        }
        cur = best;
        return MSB_OK;
    };
    // line passes, with the x passes fixed; ip: the line-pass bit of lds_inplace
    auto scan_lines = [&](int ip) -> msb_status {
        msb_launch_config best = cur;
        MSB_TRY(bn.run(cur, err) ? MSB_OK : err);
        double bt = bn.line_time();
        const int ipm = (cur.lds_inplace & ~2) | (ip << 1);
        for (int Fl : Fs) {
            for (int th : ths) {
                msb_launch_config c = cur;
                c.team_line = 0;
                c.lines_per_wg = Fl;
                c.threads_line = th;
                c.lds_inplace = ipm;
                if (bn.run(c, err) && bn.line_time() < bt) {
                    bt = bn.line_time();
                    best = c;
                }
                MSB_TRY(err);
            }
            for (int lp : lpws) {
                msb_launch_config c = cur;
                c.team_line = 1;
                c.lines_per_wg = Fl;
                c.lines_per_wave = lp;
                c.lds_inplace = ipm;
                if (bn.run(c, err) && bn.line_time() < bt) {
                    bt = bn.line_time();
                    best = c;
                }
                MSB_TRY(err);
            }
        }
        cur = best;
        return MSB_OK;
    };
    MSB_TRY(scan_x(0));
    MSB_TRY(scan_lines(0));
    // radix cap of the schedules (changes every kernel)
    {
        msb_launch_config best = cur;
        MSB_TRY(bn.run(cur, err) ? MSB_OK : err);
        double bt = bn.total();
        for (int r : {4, 8, 16}) {
            if (r == cur.max_radix) continue;
            msb_launch_config c = cur;
            c.max_radix = r;
            if (bn.run(c, err) && bn.total() < bt) {
                bt = bn.total();
                best = c;
            }
            MSB_TRY(err);
        }
        cur = best;
    }
    // in-place stages (half the LDS per workgroup: more resident workgroups, or more rows
    // or lines per workgroup), kept where they are faster; invalid candidates are skipped
    if (effort) {
        MSB_TRY(scan_x(1));
        MSB_TRY(scan_lines(1));
    }
    // the tiled single-pass product (2D): frame lengths, threads per workgroup and radix
    // caps, kept when one launch beats the tuned chain (the chain's settings stay for the
    // preconditioner and the fused solver prologues)
    if (p->dim == 2) {
        msb_launch_config best = cur;
        MSB_TRY(bn.run(cur, err) ? MSB_OK : err);
        double bt = bn.total();
        const std::vector<int> tls = effort ? std::vector<int>{16, 20, 24, 30, 32, 36, 40, 48, 60, 64, 72, 80, 96}
                                            : std::vector<int>{24, 32, 40, 48, 64};
        for (int tl : tls)
            for (int th : effort ? std::vector<int>{128, 256, 512} : std::vector<int>{256})
                for (int r : {8, 16}) {
                    msb_launch_config c = cur;
                    c.tile = tl;
                    c.threads_tile = th;
                    c.max_radix = r;
                    c.tile_regs = 0;
                    if (bn.run(c, err) && bn.total() < bt) {
                        bt = bn.total();
                        best = c;
                    }
                    MSB_TRY(err);
                }
        // register-resident frames (their own thread count; no radix cap), with runs of
        // consecutive blocks per workgroup
        for (int tl : {16, 32, 64})
            for (int run : {1, 2, 3, 4, 6, 8}) {
                msb_launch_config c = cur;
                c.tile = tl;
                c.tile_regs = 1;
                c.tile_run = run;
                if (bn.run(c, err) && bn.total() < bt) {
                    bt = bn.total();
                    best = c;
                }
                MSB_TRY(err);
            }
        cur = best;
    }
    bn.nrep = std::max(bn.nrep, 5);
    MSB_CHECK(bn.run(cur, err), err != MSB_OK ? err : MSB_EINVAL, "tuned configuration rejected");
    *best_ms = bn.total();
    return MSB_OK;
}

// Tune the precisions `prec` needs; the figure of merit is the FP32 product time
// for the refined solve (its inner iterations dominate), else that precision's.
msb_status tune_all(msb_plan_s *p, msb_precision prec, int effort, hipStream_t st, double *merit) {
    double t64 = 0.0, t32 = 0.0;
    if (prec == MSB_FP64 || prec == MSB_FP32_REFINED) MSB_TRY(tune_precision<double>(p, effort, st, &t64));
    if (prec == MSB_FP32 || prec == MSB_FP32_REFINED) MSB_TRY(tune_precision<float>(p, effort, st, &t32));
    *merit = prec == MSB_FP64 ? t64 : t32;
    return MSB_OK;
}

// Up to `count` 5-smooth lengths in [n, 1.125 n].
std::vector<int64_t> smooth_candidates(int64_t n, int count) {
    std::vector<int64_t> out;
    const int64_t hi = n + n / 8;
    for (int64_t L = n; L <= hi && (int)out.size() < count; ++L) {
        int64_t m = L;
        for (int q : {2, 3, 5})
            while (m % q == 0) m /= q;
        if (m == 1) out.push_back(L);
    }
    if (out.empty()) out.push_back(next_smooth((int)n, false));
    return out;
}

}  // namespace
}  // namespace msb

using namespace msb;

static msb_status check_prec(msb_precision prec) {
    MSB_CHECK(prec == MSB_FP64 || prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    return MSB_OK;
}

extern "C" msb_status msb_plan_get_config(msb_plan p, msb_precision prec, msb_launch_config *cfg) {
    MSB_CHECK(p && cfg, MSB_EINVAL, "null argument");
    MSB_TRY(check_prec(prec));
    *cfg = p->cfg[prec == MSB_FP32 ? 1 : 0];
    return MSB_OK;
}

extern "C" msb_status msb_plan_set_config(msb_plan p, msb_precision prec, const msb_launch_config *cfg) {
    MSB_CHECK(p && cfg, MSB_EINVAL, "null argument");
    MSB_TRY(check_prec(prec));
    const bool f32 = prec == MSB_FP32;
    MSB_TRY(check_config(p, f32, *cfg));
    msb_status s = set_schedules(p, f32, cfg->max_radix);
    if (s == MSB_OK) s = ensure_tiles(p, cfg->tile);
    if (s != MSB_OK) {
        (void)set_schedules(p, f32, p->cfg[f32].max_radix);
        return s;
    }
    p->cfg[f32] = *cfg;
    return MSB_OK;
}

extern "C" msb_status msb_plan_set_lengths(msb_plan p, const int64_t *L) {
    MSB_CHECK(p && L, MSB_EINVAL, "null argument");
    return relayout(p, L);
}

extern "C" msb_status msb_plan_autotune(msb_plan p, msb_precision prec, int effort, int lengths,
                                        msb_launch_config *best, double *best_ms, void *stream) {
    MSB_CHECK(p, MSB_EINVAL, "null plan");
    MSB_CHECK(prec == MSB_FP64 || prec == MSB_FP32 || prec == MSB_FP32_REFINED, MSB_EINVAL, "bad precision");
    MSB_CHECK(effort == 0 || effort == 1, MSB_EINVAL, "effort must be 0 or 1");
    hipStream_t st = (hipStream_t)stream;
    double merit = 0.0;
    if (!lengths) {
        MSB_TRY(tune_all(p, prec, effort, st, &merit));
    } else {
        // lengths per axis: up to 3 smooth candidates in 2D, 2 in 3D (8 layouts)
        std::vector<std::vector<int64_t>> cand(3);
        for (int a = 0; a < 3; ++a)
            cand[a] = a < p->dim ? smooth_candidates(p->n[a] + p->M, p->dim == 2 ? 3 : 2) : std::vector<int64_t>{1};
        double bm = kInf;
        int64_t bestL[3] = {p->L[0], p->L[1], p->L[2]};
        msb_launch_config bc[2] = {p->cfg[0], p->cfg[1]};
        for (int64_t lx : cand[0])
            for (int64_t ly : cand[1])
                for (int64_t lz : cand[2]) {
                    const int64_t L[3] = {lx, ly, lz};
                    MSB_TRY(relayout(p, L));
                    double m = 0.0;
                    MSB_TRY(tune_all(p, prec, effort, st, &m));
                    if (m < bm) {
                        bm = m;
                        for (int a = 0; a < 3; ++a) bestL[a] = L[a];
                        bc[0] = p->cfg[0];
                        bc[1] = p->cfg[1];
                    }
                }
        MSB_TRY(relayout(p, bestL));
        for (int f = 0; f < 2; ++f) {
            MSB_TRY(set_schedules(p, f == 1, bc[f].max_radix));
            p->cfg[f] = bc[f];
        }
        merit = bm;
    }
    if (best) *best = p->cfg[prec == MSB_FP64 ? 0 : 1];
    if (best_ms) *best_ms = merit;
    return MSB_OK;
}
