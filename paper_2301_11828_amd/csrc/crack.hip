// Crack propagation: the history-dependent bond factor mu of eq. (mu).  A bond {p, q}
// breaks for good once its stretch s = (|x' + u' - x - u| - |x' - x|) / |x' - x|
// (eq. (fra:s1)) reaches the critical stretch s0; its stiffness then moves into the
// correction D^f (eq. (df)).  The paper's Phase III (Sec. 5.2) evaluates s for every
// bond each step; here that is one data-parallel pass over the nodes (each thread a
// node p and the half stencil, bonds to q = p + o > p), reading the broken set as a
// bit mask, followed by a deterministic compaction of the new breaks (per-node counts,
// one scan of the block totals, then every block writes its nodes' breaks in node and
// offset order).  The
// new pairs are merged into the plan's broken list, which rebuilds the D^f lists.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace msb {
namespace {

constexpr int kCT = 256;        // threads per block of the stretch and emit passes
constexpr int kScanT = 1024;    // threads of the one-block scan
constexpr int kMaxWords = 8;    // mask words per node: half stencils of up to 256 bonds

struct CrackWs {
    int nh = 0;                 // half-stencil offsets
    int *hoff = nullptr;        // [nh][3]
    double *thr2 = nullptr;     // [nh] ((1 + s0) |o| h)^2 of the current call
    uint8_t *count = nullptr;   // [N] new breaks per node
    int64_t *blk = nullptr;     // [nblk + 2] per-block counts, then their exclusive scan and the total;
                                // blk[nblk + 1]: the total the stretch pass accumulates (0 between calls)
    int64_t *pairs = nullptr;   // [cap][2]
    int64_t cap = 0;
    int64_t *h_total = nullptr; // pinned
    double *h_thr2 = nullptr;   // pinned [nh]
    double s0 = -1.0;           // critical stretch thr2 holds (uploaded again when it changes)
    std::vector<int> hoff_host; // [nh][3]
    std::vector<double> len;    // [nh] |o| h
};

// Half stencil: offsets o of the plan's stencil with node id p + o > p, i.e. o > 0 in
// (z, y, x) lexicographic order; sorted that way.
std::vector<int> half_stencil(const msb_plan_s *p) {
    std::vector<std::array<int, 3>> v;
    for (int i = 0; i < p->n_off; ++i) {
        const int *o = &p->off[3 * i];
        const bool pos = o[2] > 0 || (o[2] == 0 && (o[1] > 0 || (o[1] == 0 && o[0] > 0)));
        if (pos) v.push_back({o[2], o[1], o[0]});
    }
    std::sort(v.begin(), v.end());
    std::vector<int> out;
    for (auto &a : v) {
        out.push_back(a[2]);
        out.push_back(a[1]);
        out.push_back(a[0]);
    }
    return out;
}

msb_status alloc_crack_ws(msb_plan_s *p, CrackWs *w, const std::vector<int> &hoff);

msb_status get_crack_ws(msb_plan_s *p, CrackWs *&out) {
    if (p->crack_ws) {
        out = static_cast<CrackWs *>(p->crack_ws);
        return MSB_OK;
    }
    std::vector<int> hoff = half_stencil(p);
    const int nh = (int)hoff.size() / 3;
    // per-node counts are bytes: at most 255 bonds per node in the half stencil
    MSB_CHECK(nh <= 255, MSB_EUNSUPPORTED, "crack propagation supports up to 255 bonds per node "
              "in the half stencil (this horizon has %d)", nh);
    CrackWs *w = new CrackWs();
    p->crack_ws = w;
    const msb_status s = alloc_crack_ws(p, w, hoff);
    if (s != MSB_OK) {
        crack_free(p);   // a partial workspace is never reused
        return s;
    }
    out = w;
    return MSB_OK;
}

msb_status alloc_crack_ws(msb_plan_s *p, CrackWs *w, const std::vector<int> &hoff) {
    const int nh = (int)hoff.size() / 3;
    w->hoff_host = hoff;
    w->nh = nh;
    w->len.resize(nh);
    for (int k = 0; k < nh; ++k) {
        double s2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double x = hoff[3 * k + c] * p->h;
            s2 += x * x;
        }
        w->len[k] = std::sqrt(s2);
    }
    p->mu_words = std::max(1, (nh + 31) / 32);
    const size_t N = (size_t)p->N;
    const size_t nblk = (N + kCT - 1) / kCT;
    MSB_HIP(hipMalloc(&w->hoff, sizeof(int) * std::max<size_t>(1, hoff.size())));
    MSB_HIP(hipMalloc(&w->thr2, sizeof(double) * std::max(1, nh)));
    if (nh) MSB_HIP(hipMemcpy(w->hoff, hoff.data(), sizeof(int) * hoff.size(), hipMemcpyHostToDevice));
    MSB_HIP(hipMalloc(&p->mu_mask, sizeof(uint32_t) * N * p->mu_words));
    MSB_HIP(hipMalloc(&w->count, N));
    MSB_HIP(hipMalloc(&w->blk, sizeof(int64_t) * (nblk + 2)));
    MSB_HIP(hipMemset(w->blk, 0, sizeof(int64_t) * (nblk + 2)));
    MSB_HIP(hipHostMalloc(&w->h_total, sizeof(int64_t)));
    MSB_HIP(hipHostMalloc(&w->h_thr2, sizeof(double) * std::max(1, nh)));
    p->mu_valid = false;
    return MSB_OK;
}

// Bit k of mask word (p, k / 32) <-> bond {p, p + half[k]} broken, from the host list.
msb_status upload_mask(msb_plan_s *p, CrackWs *w) {
    const int64_t nx = p->n[0], ny = p->n[1];
    const int M = p->M, S = 2 * M + 1;
    std::vector<int> lut((size_t)S * S * S, -1);
    for (int k = 0; k < w->nh; ++k) {
        const int *o = &w->hoff_host[3 * k];
        lut[((size_t)(o[2] + M) * S + (o[1] + M)) * S + (o[0] + M)] = k;
    }
    std::vector<uint32_t> mask((size_t)p->N * p->mu_words, 0);
    for (int64_t e = 0; e < p->n_pairs; ++e) {
        const int64_t a = p->bonds_host[2 * e], b = p->bonds_host[2 * e + 1];   // a < b
        const int64_t ia[3] = {a % nx, (a / nx) % ny, a / (nx * ny)};
        const int64_t ib[3] = {b % nx, (b / nx) % ny, b / (nx * ny)};
        const int k = lut[((size_t)(ib[2] - ia[2] + M) * S + (ib[1] - ia[1] + M)) * S + (ib[0] - ia[0] + M)];
        MSB_CHECK(k >= 0, MSB_EINVAL, "broken bond (%lld, %lld) is not in the half stencil", (long long)a,
                  (long long)b);
        mask[(size_t)a * p->mu_words + (k >> 5)] |= 1u << (k & 31);
    }
    MSB_HIP(hipMemcpy(p->mu_mask, mask.data(), sizeof(uint32_t) * mask.size(), hipMemcpyHostToDevice));
    p->mu_valid = true;
    return MSB_OK;
}

struct Grid {
    int d, nx, ny, nz, N, nh, words;
    int M;   // horizon in nodes: every half-stencil offset component is within [-M, M]
};

// The bonds {p, p + o} of the half stencil that are unbroken and break now: with
// l = |o| h and l' = |o h + u_{p+o} - u_p| (FP64 from the given displacements), the
// stretch s = (l' - l) / l of eq. (fra:s1) reaches s0 exactly when l'^2 >= ((1 + s0) l)^2
// (thr2, one value per offset), so neither a square root nor a division is needed.
// Branch-free over the offsets (a bond outside the grid or already broken reads node p
// itself and is masked out), so the loads of several bonds are in flight at once.
// nw: the new bits per mask word; returns their number.  IN: node p is at least M nodes from
// every face, so every neighbour p + o lies in the grid and no bounds are tested (the same
// arithmetic and result as the general form).
template <typename T, int D, bool IN = false>
__device__ __forceinline__ int node_breaks(const Grid &g, const T *__restrict__ u, const int *__restrict__ hoff,
                                           const double *__restrict__ thr2, const uint32_t *__restrict__ mu,
                                           int p, uint32_t (&nw)[kMaxWords], double h) {
    const int i = p % g.nx, j = (p / g.nx) % g.ny, k = p / (g.nx * g.ny);
    double up[D];
#pragma unroll
    for (int c = 0; c < D; ++c) up[c] = (double)u[(size_t)c * g.N + p];
    int cnt = 0;
    for (int wd = 0; wd < g.words; ++wd) {
        const uint32_t old = mu[(size_t)p * g.words + wd];
        uint32_t bits = 0;
        const int kend = min(g.nh, 32 * (wd + 1));
#pragma unroll 8
        for (int b = 32 * wd; b < kend; ++b) {
            const int ox = hoff[3 * b], oy = hoff[3 * b + 1], oz = hoff[3 * b + 2];
            const bool unbroken = !((old >> (b & 31)) & 1u);
            const bool ok = IN ? unbroken
                               : unbroken && (unsigned)(i + ox) < (unsigned)g.nx && (unsigned)(j + oy) < (unsigned)g.ny &&
                                     (unsigned)(k + oz) < (unsigned)g.nz;
            const int q = IN || ok ? p + (oz * g.ny + oy) * g.nx + ox : p;
            const int o3[3] = {ox, oy, oz};
            double s2 = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const double e = o3[c] * h + ((double)u[(size_t)c * g.N + q] - up[c]);
                s2 += e * e;
            }
            // both tests evaluated (no short circuit): the loads above then stay unconditional and
            // those of the unrolled bonds are in flight together
            const bool brk = ok & (s2 >= thr2[b]);
            bits |= (uint32_t)brk << (b & 31);
            cnt += (int)brk;
        }
        nw[wd] = bits;
    }
    return cnt;
}

// Exclusive block scan of one value per thread (blockDim a multiple of 64, <= 1024):
// wave shuffles, then the wave totals scanned by wave 0.  *total = the block's sum.
__device__ __forceinline__ long long block_exclusive_scan(long long x, long long *wsum, long long *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    long long inc = x;
    for (int off = 1; off < 64; off <<= 1) {
        const long long y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    if (wv == 0) {
        const long long t = lane < nw ? wsum[lane] : 0;
        long long it = t;
        for (int off = 1; off < 64; off <<= 1) {
            const long long y = __shfl_up(it, off, 64);
            if (lane >= off) it += y;
        }
        if (lane < nw) wsum[lane] = it - t;
        if (lane == nw - 1) wsum[16] = it;
    }
    __syncthreads();
    *total = wsum[16];
    return wsum[wv] + inc - x;
}

// One thread per node: count of the bonds that break now (fresh bits are not stored:
// the emit pass recomputes them for the few nodes with a break); block totals to blk, and
// the blocks with a break add theirs to blk[nblk + 1] (integer adds: the total is exact in any
// order), so that a call without breaks needs no scan.
template <typename T, int D>
__global__ __launch_bounds__(kCT) void k_stretch(Grid g, const T *__restrict__ u, const int *__restrict__ hoff,
                                                 const double *__restrict__ thr2, const uint32_t *__restrict__ mu,
                                                 uint8_t *__restrict__ count, int64_t *__restrict__ blk, double h) {
    __shared__ int red[kCT / 64];
    const int p = blockIdx.x * kCT + threadIdx.x;
    int cnt = 0;
    if (p < g.N) {
        uint32_t nw[kMaxWords];
        // a wave whose nodes are all at least M from every face takes the form without bounds
        // tests (the branch is uniform across the wave)
        const int i = p % g.nx, j = (p / g.nx) % g.ny, k = p / (g.nx * g.ny);
        const bool in = i >= g.M && i < g.nx - g.M && j >= g.M && j < g.ny - g.M &&
                        (D == 2 || (k >= g.M && k < g.nz - g.M));
        if (__all(in))
            cnt = node_breaks<T, D, true>(g, u, hoff, thr2, mu, p, nw, h);
        else
            cnt = node_breaks<T, D>(g, u, hoff, thr2, mu, p, nw, h);
        count[p] = (uint8_t)cnt;
    }
    int v = cnt;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int wv = 0; wv < kCT / 64; ++wv) t += red[wv];
        blk[blockIdx.x] = t;
        if (t) atomicAdd(reinterpret_cast<unsigned long long *>(blk + gridDim.x + 1), (unsigned long long)t);
    }
}

// Exclusive scan of blk[0..n) in place, blk[n] = total; one block, each thread a
// contiguous run of ceil(n / kScanT) values.
__global__ __launch_bounds__(kScanT) void k_scan(int64_t *blk, int n) {
    __shared__ long long wsum[17];
    const int per = (n + kScanT - 1) / kScanT;
    const int b0 = min(n, threadIdx.x * per), b1 = min(n, b0 + per);
    long long s = 0;
    for (int i = b0; i < b1; ++i) s += blk[i];
    long long total = 0;
    long long run = block_exclusive_scan(s, wsum, &total);
    for (int i = b0; i < b1; ++i) {
        const long long x = blk[i];
        blk[i] = run;
        run += x;
    }
    if (threadIdx.x == 0) blk[n] = total;
}

// Every block writes its nodes' new breaks (p, p + o) from offset blk[block] on, in
// node order and, per node, in half-stencil order, and marks them broken in mu.  A node
// writes exactly count[p] entries (fewer found would leave (-1, -1), which the host
// rejects), so the writes stay inside the scanned range.
template <typename T, int D>
__global__ __launch_bounds__(kCT) void k_emit(Grid g, const T *__restrict__ u, const int *__restrict__ hoff,
                                              const double *__restrict__ thr2, uint32_t *__restrict__ mu,
                                              const uint8_t *__restrict__ count, const int64_t *__restrict__ blk,
                                              int64_t *__restrict__ pairs, double h) {
    __shared__ long long wsum[17];
    const int p = blockIdx.x * kCT + threadIdx.x;
    const int c = p < g.N ? count[p] : 0;
    long long total = 0;
    const long long off = block_exclusive_scan(c, wsum, &total);
    if (c == 0) return;
    uint32_t nw[kMaxWords];
    node_breaks<T, D>(g, u, hoff, thr2, mu, p, nw, h);
    int64_t at = blk[blockIdx.x] + off;
    const int64_t end = at + c;
    for (int wd = 0; wd < g.words; ++wd) {
        const uint32_t bits = nw[wd];
        if (!bits) continue;
        mu[(size_t)p * g.words + wd] |= bits;
        for (int b = 0; b < 32 && at < end; ++b) {
            if (!((bits >> b) & 1u)) continue;
            const int kk = 32 * wd + b;
            pairs[2 * at] = p;
            pairs[2 * at + 1] = p + (hoff[3 * kk + 2] * g.ny + hoff[3 * kk + 1]) * g.nx + hoff[3 * kk];
            ++at;
        }
    }
    for (; at < end; ++at) {
        pairs[2 * at] = -1;
        pairs[2 * at + 1] = -1;
    }
}

template <typename T>
msb_status crack_update_t(msb_plan_s *p, const T *u, double s0, int64_t *n_new, hipStream_t st) {
    CrackWs *w = nullptr;
    MSB_TRY(get_crack_ws(p, w));
    if (!p->mu_valid) MSB_TRY(upload_mask(p, w));
    *n_new = 0;
    if (w->nh == 0) return MSB_OK;
    if (s0 != w->s0) {
        for (int k = 0; k < w->nh; ++k) {
            const double l = (1.0 + s0) * w->len[k];
            w->h_thr2[k] = l * l;
        }
        MSB_HIP(hipMemcpyAsync(w->thr2, w->h_thr2, sizeof(double) * w->nh, hipMemcpyHostToDevice, st));
        w->s0 = s0;
    }
    const Grid g{p->dim, (int)p->n[0], (int)p->n[1], (int)p->n[2], (int)p->N, w->nh, p->mu_words, p->M};
    const int nblk = (int)((p->N + kCT - 1) / kCT);
    if (p->dim == 2)
        hipLaunchKernelGGL((k_stretch<T, 2>), dim3(nblk), dim3(kCT), 0, st, g, u, (const int *)w->hoff,
                           (const double *)w->thr2, (const uint32_t *)p->mu_mask, w->count, w->blk, p->h);
    else
        hipLaunchKernelGGL((k_stretch<T, 3>), dim3(nblk), dim3(kCT), 0, st, g, u, (const int *)w->hoff,
                           (const double *)w->thr2, (const uint32_t *)p->mu_mask, w->count, w->blk, p->h);
    MSB_HIP(hipGetLastError());
    MSB_HIP(hipMemcpyAsync(w->h_total, w->blk + nblk + 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    const int64_t total = *w->h_total;
    if (total == 0) return MSB_OK;
    // breaks: the running total back to 0 for the next call, then the block offsets
    MSB_HIP(hipMemsetAsync(w->blk + nblk + 1, 0, sizeof(int64_t), st));
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanT), 0, st, w->blk, nblk);
    MSB_HIP(hipGetLastError());
    if (total > w->cap) {
        if (w->pairs) MSB_HIP(hipFree(w->pairs));
        w->pairs = nullptr;
        w->cap = 0;
        MSB_HIP(hipMalloc(&w->pairs, sizeof(int64_t) * 2 * total));
        w->cap = total;
    }
    if (p->dim == 2)
        hipLaunchKernelGGL((k_emit<T, 2>), dim3(nblk), dim3(kCT), 0, st, g, u, (const int *)w->hoff,
                           (const double *)w->thr2, p->mu_mask, (const uint8_t *)w->count, (const int64_t *)w->blk,
                           w->pairs, p->h);
    else
        hipLaunchKernelGGL((k_emit<T, 3>), dim3(nblk), dim3(kCT), 0, st, g, u, (const int *)w->hoff,
                           (const double *)w->thr2, p->mu_mask, (const uint8_t *)w->count, (const int64_t *)w->blk,
                           w->pairs, p->h);
    MSB_HIP(hipGetLastError());
    std::vector<int64_t> fresh((size_t)2 * total);
    MSB_HIP(hipMemcpyAsync(fresh.data(), w->pairs, sizeof(int64_t) * 2 * total, hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    // merge into the sorted broken list (both sorted by (p, q) after sorting the new ones)
    std::vector<std::pair<int64_t, int64_t>> nv((size_t)total);
    for (int64_t e = 0; e < total; ++e) {
        nv[e] = {fresh[2 * e], fresh[2 * e + 1]};
        if (nv[e].first < 0) {
            p->mu_valid = false;
            MSB_CHECK(false, MSB_EDEVICE, "crack update: the emit pass disagreed with the count pass");
        }
    }
    std::sort(nv.begin(), nv.end());
    const std::vector<int64_t> &old = p->bonds_host;
    std::vector<int64_t> merged;
    merged.reserve(old.size() + fresh.size());
    size_t a = 0, b = 0;
    const size_t na = old.size() / 2;
    while (a < na || b < nv.size()) {
        const bool take_old = b == nv.size() ||
                              (a < na && std::make_pair(old[2 * a], old[2 * a + 1]) < nv[b]);
        if (take_old) {
            merged.push_back(old[2 * a]);
            merged.push_back(old[2 * a + 1]);
            ++a;
        } else {
            merged.push_back(nv[b].first);
            merged.push_back(nv[b].second);
            ++b;
        }
    }
    msb_status s = set_bonds_impl(p, merged.data(), (int64_t)(merged.size() / 2));
    if (s != MSB_OK) {
        p->mu_valid = false;   // the mask already holds the new breaks
        return s;
    }
    *n_new = total;
    return MSB_OK;
}

}  // namespace

void crack_free(msb_plan_s *p) {
    CrackWs *w = static_cast<CrackWs *>(p->crack_ws);
    if (w) {
        void *b[] = {w->hoff, w->thr2, w->count, w->blk, w->pairs};
        for (void *x : b)
            if (x) (void)hipFree(x);
        if (w->h_total) (void)hipHostFree(w->h_total);
        if (w->h_thr2) (void)hipHostFree(w->h_thr2);
        delete w;
        p->crack_ws = nullptr;
    }
    if (p->mu_mask) (void)hipFree(p->mu_mask);
    p->mu_mask = nullptr;
    p->mu_valid = false;
}

}  // namespace msb

using namespace msb;

extern "C" msb_status msb_crack_update(msb_plan p, msb_precision prec, const void *u, double s0, int64_t *n_new,
                                       void *stream) {
    MSB_CHECK(p, MSB_EINVAL, "null plan");
    MSB_CHECK(u && n_new, MSB_EINVAL, "null argument");
    MSB_CHECK(p->B == 1, MSB_EUNSUPPORTED, "crack propagation needs a single-case plan (batch %d)", p->B);
    MSB_CHECK(std::isfinite(s0) && s0 > 0.0, MSB_EINVAL, "critical stretch must be finite and > 0");
    MSB_CHECK(p->N <= (int64_t)INT32_MAX / 2, MSB_EINVAL, "grid too large for crack propagation");
    int dev = -1;
    MSB_HIP(hipGetDevice(&dev));
    MSB_CHECK(dev == p->device, MSB_EINVAL, "plan was created on device %d, current is %d", p->device, dev);
    hipStream_t st = (hipStream_t)stream;
    if (prec == MSB_FP64) return crack_update_t<double>(p, (const double *)u, s0, n_new, st);
    MSB_CHECK(prec == MSB_FP32, MSB_EINVAL, "precision must be MSB_FP64 or MSB_FP32");
    return crack_update_t<float>(p, (const float *)u, s0, n_new, st);
}
