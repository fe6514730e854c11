// Crack propagation: the history-dependent bond factor mu of eq. (mu).  A bond {p, q}
// breaks for good once its stretch s = (|x' + u' - x - u| - |x' - x|) / |x' - x|
// (eq. (fra:s1)) reaches the critical stretch s0; its stiffness then moves into the
// correction D^f (eq. (df)).  The paper's Phase III (Sec. 5.2) evaluates s for every
// bond each step; here that is one data-parallel pass over the nodes (each thread a
// node p and the half stencil, bonds to q = p + o > p), reading the broken set as a
// bit mask, followed by a deterministic compaction of the new breaks (per-block counts,
// one scan, then every block writes its nodes' breaks in node and offset order).  The
// new pairs are merged into the plan's broken list, which rebuilds the D^f lists.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace msb {
namespace {

constexpr int kCT = 256;   // threads per block of the stretch and emit passes

struct CrackWs {
    int nh = 0;                 // half-stencil offsets
    int *hoff = nullptr;        // [nh][3]
    double *hlen = nullptr;     // [nh] |o| h
    uint64_t *fresh = nullptr;  // [N][words] bonds that break in this update
    int *count = nullptr;       // [N] new breaks per node
    int64_t *blk = nullptr;     // [nblk + 1] per-block counts, then their exclusive scan
    int64_t *pairs = nullptr;   // [cap][2]
    int64_t cap = 0;
    int64_t *h_total = nullptr; // pinned
    std::vector<int> hoff_host; // [nh][3]
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

msb_status get_crack_ws(msb_plan_s *p, CrackWs *&out) {
    if (p->crack_ws) {
        out = static_cast<CrackWs *>(p->crack_ws);
        return MSB_OK;
    }
    CrackWs *w = new CrackWs();
    p->crack_ws = w;
    w->hoff_host = half_stencil(p);
    w->nh = (int)w->hoff_host.size() / 3;
    std::vector<double> len(w->nh);
    for (int k = 0; k < w->nh; ++k) {
        double s2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double x = w->hoff_host[3 * k + c] * p->h;
            s2 += x * x;
        }
        len[k] = std::sqrt(s2);
    }
    p->mu_words = std::max(1, (w->nh + 63) / 64);
    const size_t N = (size_t)p->N;
    const size_t nblk = (N + kCT - 1) / kCT;
    MSB_HIP(hipMalloc(&w->hoff, sizeof(int) * std::max<size_t>(1, w->hoff_host.size())));
    MSB_HIP(hipMalloc(&w->hlen, sizeof(double) * std::max(1, w->nh)));
    if (w->nh) {
        MSB_HIP(hipMemcpy(w->hoff, w->hoff_host.data(), sizeof(int) * w->hoff_host.size(), hipMemcpyHostToDevice));
        MSB_HIP(hipMemcpy(w->hlen, len.data(), sizeof(double) * w->nh, hipMemcpyHostToDevice));
    }
    MSB_HIP(hipMalloc(&p->mu_mask, sizeof(uint64_t) * N * p->mu_words));
    MSB_HIP(hipMalloc(&w->fresh, sizeof(uint64_t) * N * p->mu_words));
    MSB_HIP(hipMalloc(&w->count, sizeof(int) * N));
    MSB_HIP(hipMalloc(&w->blk, sizeof(int64_t) * (nblk + 1)));
    MSB_HIP(hipHostMalloc(&w->h_total, sizeof(int64_t)));
    p->mu_valid = false;
    out = w;
    return MSB_OK;
}

// Bit k of mask word (p, k / 64) <-> bond {p, p + half[k]} broken, from the host list.
msb_status upload_mask(msb_plan_s *p, CrackWs *w) {
    const int64_t nx = p->n[0], ny = p->n[1];
    const int M = p->M, S = 2 * M + 1;
    std::vector<int> lut((size_t)S * S * S, -1);
    for (int k = 0; k < w->nh; ++k) {
        const int *o = &w->hoff_host[3 * k];
        lut[((size_t)(o[2] + M) * S + (o[1] + M)) * S + (o[0] + M)] = k;
    }
    std::vector<uint64_t> mask((size_t)p->N * p->mu_words, 0);
    for (int64_t e = 0; e < p->n_pairs; ++e) {
        const int64_t a = p->bonds_host[2 * e], b = p->bonds_host[2 * e + 1];   // a < b
        const int64_t ia[3] = {a % nx, (a / nx) % ny, a / (nx * ny)};
        const int64_t ib[3] = {b % nx, (b / nx) % ny, b / (nx * ny)};
        const int k = lut[((size_t)(ib[2] - ia[2] + M) * S + (ib[1] - ia[1] + M)) * S + (ib[0] - ia[0] + M)];
        MSB_CHECK(k >= 0, MSB_EINVAL, "broken bond (%lld, %lld) is not in the half stencil", (long long)a,
                  (long long)b);
        mask[(size_t)a * p->mu_words + (k >> 6)] |= 1ull << (k & 63);
    }
    MSB_HIP(hipMemcpy(p->mu_mask, mask.data(), sizeof(uint64_t) * mask.size(), hipMemcpyHostToDevice));
    p->mu_valid = true;
    return MSB_OK;
}

struct Grid {
    int d, nx, ny, nz, N, nh, words;
    double h, s0;
};

// One thread per node p: the stretch of every unbroken bond {p, p + o} of the half
// stencil (FP64 from the given displacements); fresh = bonds with s >= s0, count =
// their number, blk = the block's total.
template <typename T>
__global__ __launch_bounds__(kCT) void k_stretch(Grid g, const T *__restrict__ u, const int *__restrict__ hoff,
                                                 const double *__restrict__ hlen, const uint64_t *__restrict__ mu,
                                                 uint64_t *__restrict__ fresh, int *__restrict__ count,
                                                 int64_t *__restrict__ blk) {
    __shared__ int red[kCT / 64];
    const int p = blockIdx.x * kCT + threadIdx.x;
    int cnt = 0;
    if (p < g.N) {
        const int i = p % g.nx, j = (p / g.nx) % g.ny, k = p / (g.nx * g.ny);
        double up[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < g.d; ++c) up[c] = (double)u[(size_t)c * g.N + p];
        for (int wd = 0; wd < g.words; ++wd) {
            const uint64_t old = mu[(size_t)p * g.words + wd];
            uint64_t nw = 0;
            const int kend = min(g.nh, 64 * (wd + 1));
            for (int b = 64 * wd; b < kend; ++b) {
                if ((old >> (b & 63)) & 1ull) continue;
                const int ox = hoff[3 * b], oy = hoff[3 * b + 1], oz = hoff[3 * b + 2];
                const int ii = i + ox, jj = j + oy, kk = k + oz;
                if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) continue;
                const int q = p + (oz * g.ny + oy) * g.nx + ox;
                const int o3[3] = {ox, oy, oz};
                double s2 = 0.0;
                for (int c = 0; c < g.d; ++c) {
                    const double e = o3[c] * g.h + ((double)u[(size_t)c * g.N + q] - up[c]);
                    s2 += e * e;
                }
                const double s = (sqrt(s2) - hlen[b]) / hlen[b];
                if (s >= g.s0) {
                    nw |= 1ull << (b & 63);
                    ++cnt;
                }
            }
            fresh[(size_t)p * g.words + wd] = nw;
        }
        count[p] = cnt;
    }
    // block total (the wave sums, then wave 0 adds them)
    int v = cnt;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int wv = 0; wv < kCT / 64; ++wv) t += red[wv];
        blk[blockIdx.x] = t;
    }
}

// Exclusive scan of blk[0..n) in place, blk[n] = total; one block of kCT threads,
// chunks of kCT with a running carry.
__global__ __launch_bounds__(kCT) void k_scan(int64_t *blk, int n) {
    __shared__ int64_t s[kCT];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += kCT) {
        const int i = base + threadIdx.x;
        const int64_t x = i < n ? blk[i] : 0;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < kCT; off <<= 1) {   // Hillis-Steele inclusive scan
            const int64_t y = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        const int64_t c0 = carry;
        if (i < n) blk[i] = c0 + s[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == kCT - 1) carry = c0 + s[kCT - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) blk[n] = carry;
}

// Every block writes its nodes' new breaks (p, p + o) from offset blk[block] on, in
// node order and, per node, in half-stencil order; and marks them broken in mu.
__global__ __launch_bounds__(kCT) void k_emit(Grid g, const int *__restrict__ hoff, const int *__restrict__ count,
                                              const uint64_t *__restrict__ fresh, uint64_t *__restrict__ mu,
                                              const int64_t *__restrict__ blk, int64_t *__restrict__ pairs) {
    __shared__ int s[kCT];
    const int p = blockIdx.x * kCT + threadIdx.x;
    const int c = p < g.N ? count[p] : 0;
    s[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kCT; off <<= 1) {
        const int y = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    if (p >= g.N || c == 0) return;
    int64_t at = blk[blockIdx.x] + s[threadIdx.x] - c;
    for (int wd = 0; wd < g.words; ++wd) {
        const uint64_t nw = fresh[(size_t)p * g.words + wd];
        if (!nw) continue;
        mu[(size_t)p * g.words + wd] |= nw;
        for (int b = 0; b < 64; ++b) {
            if (!((nw >> b) & 1ull)) continue;
            const int kk = 64 * wd + b;
            const int q = p + (hoff[3 * kk + 2] * g.ny + hoff[3 * kk + 1]) * g.nx + hoff[3 * kk];
            pairs[2 * at] = p;
            pairs[2 * at + 1] = q;
            ++at;
        }
    }
}

template <typename T>
msb_status crack_update_t(msb_plan_s *p, const T *u, double s0, int64_t *n_new, hipStream_t st) {
    CrackWs *w = nullptr;
    MSB_TRY(get_crack_ws(p, w));
    if (!p->mu_valid) MSB_TRY(upload_mask(p, w));
    *n_new = 0;
    if (w->nh == 0) return MSB_OK;
    const Grid g{p->dim, (int)p->n[0], (int)p->n[1], (int)p->n[2], (int)p->N, w->nh, p->mu_words, p->h, s0};
    const int nblk = (int)((p->N + kCT - 1) / kCT);
    hipLaunchKernelGGL(k_stretch<T>, dim3(nblk), dim3(kCT), 0, st, g, u, (const int *)w->hoff,
                       (const double *)w->hlen, (const uint64_t *)p->mu_mask, w->fresh, w->count, w->blk);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kCT), 0, st, w->blk, nblk);
    MSB_HIP(hipGetLastError());
    MSB_HIP(hipMemcpyAsync(w->h_total, w->blk + nblk, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    const int64_t total = *w->h_total;
    if (total == 0) return MSB_OK;
    if (total > w->cap) {
        if (w->pairs) MSB_HIP(hipFree(w->pairs));
        w->pairs = nullptr;
        w->cap = 0;
        MSB_HIP(hipMalloc(&w->pairs, sizeof(int64_t) * 2 * total));
        w->cap = total;
    }
    hipLaunchKernelGGL(k_emit, dim3(nblk), dim3(kCT), 0, st, g, (const int *)w->hoff, (const int *)w->count,
                       (const uint64_t *)w->fresh, p->mu_mask, (const int64_t *)w->blk, w->pairs);
    MSB_HIP(hipGetLastError());
    std::vector<int64_t> fresh((size_t)2 * total);
    MSB_HIP(hipMemcpyAsync(fresh.data(), w->pairs, sizeof(int64_t) * 2 * total, hipMemcpyDeviceToHost, st));
    MSB_HIP(hipStreamSynchronize(st));
    // merge into the sorted broken list (both sorted by (p, q) after sorting the new ones)
    std::vector<std::pair<int64_t, int64_t>> nv((size_t)total);
    for (int64_t e = 0; e < total; ++e) nv[e] = {fresh[2 * e], fresh[2 * e + 1]};
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
        void *b[] = {w->hoff, w->hlen, w->fresh, w->count, w->blk, w->pairs};
        for (void *x : b)
            if (x) (void)hipFree(x);
        if (w->h_total) (void)hipHostFree(w->h_total);
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
