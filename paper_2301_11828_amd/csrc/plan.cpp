// Plan creation: everything the FFT product needs that does not change between
// products (the paper's "matrix assembly" phase, Sec. 5.1):
//   * the stencil of bond weights W^{ab}(o) of eq. (frb:e1) / (thm:e2), with the
//     partial-volume factor of eq. (fac:e1) and an optional radial influence;
//   * the kernel tensor K (centre = minus the sum of all bond weights, eq. (frb:e4))
//     wrapped into the generating array G (Sec. 3.3 for 2D, Sec. 4 for 3D) and its
//     spectrum, which is real because K is even in every component;
//   * the incomplete-horizon diagonal D^e of eq. (mat:se) as a table indexed by the
//     node's clamped distances to the grid faces;
//   * the broken-bond lists of eq. (df), grouped per grid row;
//   * the per-DOF constraint mask of Sec. 3.4 / Remark 2;
//   * FFT schedules and twiddles, and device workspace.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <functional>
#include <thread>
#include <numeric>

#include "common.hpp"

namespace msb {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

// ------------------------------------------------------------------ lengths
// Radices the device code implements: basic 2, 3, 4, 5, 8 and register-composite
// 6, 9, 10, 12, 15, 16 (two-level Cooley-Tukey inside a thread; kernels built for
// radix <= 16 only instantiate these).
static const int kRadices[] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};

// Default radix caps (measured: FP64 kernels keep more occupancy with the basic
// radices, FP32 gains from fewer LDS stages); the launch configuration can change them.
constexpr int kDefaultMaxRadix64 = 8, kDefaultMaxRadix32 = 16;

// Factor L into the fewest Stockham stages with radix <= rmax; ties go to the
// factorisation whose smallest radix is largest (balanced stages).
bool factor_length(int L, std::vector<int> &radices, int rmax_in) {
    radices.clear();
    {
        int n = L;
        for (int p : {2, 3, 5})
            while (n % p == 0) n /= p;
        if (n != 1) return false;
    }
    if (L == 1) {
        radices.push_back(1);
        return true;
    }
    const int rmax = std::max(2, rmax_in);
    // best[n] = (stages, -min radix) over factorisations of n
    std::vector<int> st(L + 1, 1 << 20), mn(L + 1, 0), pick(L + 1, 0);
    st[1] = 0;
    mn[1] = 1 << 20;
    for (int n = 2; n <= L; ++n) {
        if (L % n) continue;
        for (int r : kRadices) {
            if ((r > rmax && r != 5) || n % r) continue;   // 5 is a basic radix under every cap
            const int m = n / r;
            if (st[m] >= (1 << 20)) continue;
            const int s = st[m] + 1, lo = std::min(mn[m], r);
            if (s < st[n] || (s == st[n] && lo > mn[n])) {
                st[n] = s;
                mn[n] = lo;
                pick[n] = r;
            }
        }
    }
    if (st[L] >= (1 << 20)) return false;
    for (int n = L; n > 1; n /= pick[n]) radices.push_back(pick[n]);
    std::sort(radices.begin(), radices.end(), std::greater<int>());
    return true;
}

int next_smooth(int nmin, bool even_only) {
    for (int L = std::max(nmin, 1);; ++L) {
        if (even_only && (L & 1) && L > 1) continue;
        int n = L;
        for (int p : {2, 3, 5})
            while (n % p == 0) n /= p;
        if (n == 1) return L;
    }
}

int64_t rows_total(const msb_plan_s *p) { return p->n[1] * p->n[2]; }

static int comp_index(int a, int b, int d) {
    if (a > b) std::swap(a, b);
    if (d == 2) return a == 0 ? b : 2;                       // xx xy yy
    static const int t[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};  // xx xy xz yy yz zz
    return t[a][b];
}

size_t spectrum_len(const msb_plan_s *p) { return (size_t)p->H * p->L[1] * p->L[2]; }

// cos/sin(2 pi t / L), t in [0, L), long double, argument reduced to the first octant.
static void unit_circle(int L, std::vector<long double> &c, std::vector<long double> &s) {
    c.resize(L);
    s.resize(L);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int t = 0; t < L; ++t) {
        // angle = 2 pi t / L; reduce with exact integer arithmetic on 8t vs L
        long long t8 = 8LL * t;
        int oct = (int)(t8 / L);              // octant 0..7
        long long rem = t8 - (long long)oct * L;  // in [0, L)
        long double th = pi / 4 * (long double)rem / (long double)L;  // in [0, pi/4)
        long double cs = cosl(th), sn = sinl(th);
        long double cv = 0, sv = 0;
        switch (oct) {   // angle = oct*pi/4 + th
            case 0: cv = cs; sv = sn; break;
            case 1: { long double a = pi / 4 - th; cv = sinl(a); sv = cosl(a); break; }
            case 2: cv = -sn; sv = cs; break;
            case 3: { long double a = pi / 4 - th; cv = -cosl(a); sv = sinl(a); break; }
            case 4: cv = -cs; sv = -sn; break;
            case 5: { long double a = pi / 4 - th; cv = -sinl(a); sv = -cosl(a); break; }
            case 6: cv = sn; sv = -cs; break;
            default: { long double a = pi / 4 - th; cv = cosl(a); sv = -sinl(a); break; }
        }
        c[t] = cv;
        s[t] = sv;
    }
}

static msb_status axis_schedule(FftAxis &ax, bool fp32, int max_radix) {
    std::vector<int> r;
    MSB_CHECK(factor_length(ax.L, r, max_radix), MSB_EINVAL, "FFT length %d is not 5-smooth", ax.L);
    MSB_CHECK((int)r.size() <= kMaxPasses, MSB_EINVAL, "FFT length %d needs too many stages", ax.L);
    const int np = ax.L == 1 ? 0 : (int)r.size();
    int *dst = fp32 ? ax.radix32 : ax.radix;
    for (int i = 0; i < kMaxPasses; ++i) dst[i] = i < np ? r[i] : 0;
    (fp32 ? ax.np32 : ax.np) = np;
    return MSB_OK;
}

FftSched make_sched(const FftAxis &ax, bool fp32, int max_radix) {
    FftAxis t = ax;
    if (axis_schedule(t, fp32, max_radix) != MSB_OK) return sched_of(ax, fp32);
    return sched_of(t, fp32);
}

msb_status set_schedules(msb_plan_s *p, bool fp32, int max_radix) {
    for (int a = 0; a < 3; ++a) MSB_TRY(axis_schedule(p->ax[a], fp32, max_radix));
    return MSB_OK;
}

static msb_status make_axis(int L, FftAxis &ax) {
    ax.L = L;
    MSB_TRY(axis_schedule(ax, false, kDefaultMaxRadix64));
    MSB_TRY(axis_schedule(ax, true, kDefaultMaxRadix32));
    std::vector<long double> c, s;
    unit_circle(L, c, s);
    std::vector<double2> t64(L);
    std::vector<float2> t32(L);
    for (int t = 0; t < L; ++t) {
        t64[t].x = (double)c[t];
        t64[t].y = -(double)s[t];
        t32[t].x = (float)c[t];
        t32[t].y = -(float)s[t];
    }
    MSB_HIP(hipMalloc(&ax.tw64, sizeof(double2) * L));
    MSB_HIP(hipMalloc(&ax.tw32, sizeof(float2) * L));
    MSB_HIP(hipMemcpy(ax.tw64, t64.data(), sizeof(double2) * L, hipMemcpyHostToDevice));
    MSB_HIP(hipMemcpy(ax.tw32, t32.data(), sizeof(float2) * L, hipMemcpyHostToDevice));
    return MSB_OK;
}

// ------------------------------------------------------------------ stencil
// Offsets o with 0 < |o|^2 <= M^2 (horizon membership decided on integers, delta = M h).
static void build_offsets(msb_plan_s *p) {
    const int M = p->M;
    const int Mz = p->dim == 3 ? M : 0;
    p->off.clear();
    for (int oz = -Mz; oz <= Mz; ++oz)
        for (int oy = -M; oy <= M; ++oy)
            for (int ox = -M; ox <= M; ++ox) {
                int s2 = ox * ox + oy * oy + oz * oz;
                if (s2 == 0 || s2 > M * M) continue;
                p->off.push_back(ox);
                p->off.push_back(oy);
                p->off.push_back(oz);
            }
    p->n_off = (int)p->off.size() / 3;
}

// W^{c}(o) for every offset (index units of eq. (frb:e1)/(thm:e2)):
//   alpha * omega(|o|/M) * lambda(|o|) * h^(d-1) * o_a o_b / |o|^3,
//   lambda = 1 for |o|^2 <= M^2 - M (|xi| <= delta - h/2), else M + 1/2 - |o| (eq. (fac:e1)).
static void bond_weights(const msb_plan_s *p, const std::vector<double> &infl,
                         std::vector<long double> &W) {
    const int d = p->dim, M = p->M, nc = p->ncomp;
    W.assign((size_t)nc * p->n_off, 0.0L);
    long double hp = 1.0L;
    for (int a = 0; a < d - 1; ++a) hp *= p->h;
    for (int i = 0; i < p->n_off; ++i) {
        const int *o = &p->off[3 * i];
        long long s2 = (long long)o[0] * o[0] + (long long)o[1] * o[1] + (long long)o[2] * o[2];
        long double r = sqrtl((long double)s2);
        long double lam = (s2 <= (long long)M * M - M) ? 1.0L : (M + 0.5L - r);
        long double om = 1.0L;
        if (!infl.empty()) {
            om = 0.0L;
            long double x = r / M, xp = 1.0L;
            for (size_t k = 0; k < infl.size(); ++k) {
                om += (long double)infl[k] * xp;
                xp *= x;
            }
        }
        long double c = (long double)p->alpha * om * lam * hp / (r * r * r);
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b)
                W[(size_t)comp_index(a, b, d) * p->n_off + i] = c * (long double)o[a] * o[b];
    }
}

// Spectrum of the generating array, component by component (Sec. 3.3 / Sec. 4):
// G[o mod L] = K(o), so G_hat(k) = sum_o K(o) exp(-2 pi i k.o/L).  K^{ab} is even
// in every axis for a == b and odd in axes a, b (even in the third) otherwise, so
// G_hat = sign * sum_o K(o) prod_axis phi_axis(2 pi k o / L) with phi = cos on even
// axes, sin on odd axes and sign = -1 for a != b: real.  Evaluated axis by axis.
// Output layout [comp][kx < H][ky < Ly][kz < Lz], scaled by 1/(Lx Ly Lz).
// Rows of the exact unit circle for offsets m = -Mo..Mo along one axis:
// row[(m + Mo) * L + k] = cos (or sin when odd) of 2 pi k m / L, rounded to double.
static void offset_rows(int L, int Mo, bool odd, const std::vector<long double> &c,
                        const std::vector<long double> &sn, std::vector<double> &row) {
    row.resize((size_t)(2 * Mo + 1) * L);
    for (int m = -Mo; m <= Mo; ++m)
        for (int k = 0; k < L; ++k) {
            long long t = ((long long)k * m) % L;
            if (t < 0) t += L;
            row[(size_t)(m + Mo) * L + k] = (double)(odd ? sn[t] : c[t]);
        }
}

// Real spectra of the generating arrays (Sec. 3.3 and Sec. 4): G^{ab} is the stencil
// K^{ab}(o) placed at o mod L, so its DFT is the separable sum over the (2M+1)^d box
// of K(o) e^{-2 pi i k.o / L}.  K is even in every coordinate for a = b and odd in
// x_a and x_b for a != b, so each axis contributes a cosine or a sine (the product of
// the two sines of an odd pair gives the factor -1).  Computed axis by axis in double
// from the exact unit circle; scaled by 1 / prod(L) (the inverse transform's factor).
static void build_spectrum(const msb_plan_s *p, const std::vector<long double> &W,
                           std::vector<double> &spec) {
    const int d = p->dim, M = p->M, nc = p->ncomp;
    const int Bx = 2 * M + 1, By = 2 * M + 1, Bz = d == 3 ? 2 * M + 1 : 1;
    const int Mz = d == 3 ? M : 0;
    const int H = (int)p->H, Ly = (int)p->L[1], Lz = (int)p->L[2], Lx = (int)p->L[0];
    std::vector<long double> cx, sx, cy, sy, cz, sz;
    unit_circle(Lx, cx, sx);
    unit_circle(Ly, cy, sy);
    unit_circle(Lz, cz, sz);
    std::vector<double> rx[2], ry[2], rz[2];   // [even, odd]
    for (int o = 0; o < 2; ++o) {
        offset_rows(Lx, M, o == 1, cx, sx, rx[o]);
        offset_rows(Ly, M, o == 1, cy, sy, ry[o]);
        offset_rows(Lz, Mz, o == 1, cz, sz, rz[o]);
    }
    const double scale = (double)(1.0L / ((long double)Lx * Ly * Lz));
    spec.assign((size_t)nc * H * Ly * Lz, 0.0);

    std::vector<double> K((size_t)Bz * By * Bx);
    std::vector<double> S1((size_t)Bz * By * H), S2((size_t)Bz * H * Ly);
    for (int a = 0; a < d; ++a)
        for (int b = a; b < d; ++b) {
            const int c = comp_index(a, b, d);
            std::fill(K.begin(), K.end(), 0.0);
            long double centre = 0.0L;
            for (int i = 0; i < p->n_off; ++i) {
                const int *o = &p->off[3 * i];
                const long double w = W[(size_t)c * p->n_off + i];
                K[((size_t)(o[2] + Mz) * By + (o[1] + M)) * Bx + (o[0] + M)] = (double)w;
                centre -= w;
            }
            K[((size_t)Mz * By + M) * Bx + M] = (double)centre;   // eq. (frb:e4)
            const int oddx = (a != b) && (a == 0 || b == 0);
            const int oddy = (a != b) && (a == 1 || b == 1);
            const int oddz = (a != b) && (a == 2 || b == 2);
            const double sign = (a != b) ? -1.0 : 1.0;
            // stage x: S1[z][y][kx] = sum_x K[z][y][x] row_x[x][kx]
            std::fill(S1.begin(), S1.end(), 0.0);
            for (int z = 0; z < Bz; ++z)
                for (int y = 0; y < By; ++y) {
                    double *dst = &S1[((size_t)z * By + y) * H];
                    for (int x = 0; x < Bx; ++x) {
                        const double k = K[((size_t)z * By + y) * Bx + x];
                        if (k == 0.0) continue;
                        const double *row = &rx[oddx][(size_t)x * Lx];
                        for (int kx = 0; kx < H; ++kx) dst[kx] += k * row[kx];
                    }
                }
            // stage y: S2[z][kx][ky] = sum_y S1[z][y][kx] row_y[y][ky]
            std::fill(S2.begin(), S2.end(), 0.0);
            for (int z = 0; z < Bz; ++z)
                for (int kx = 0; kx < H; ++kx) {
                    double *dst = &S2[((size_t)z * H + kx) * Ly];
                    for (int y = 0; y < By; ++y) {
                        const double s1 = S1[((size_t)z * By + y) * H + kx];
                        if (s1 == 0.0) continue;
                        const double *row = &ry[oddy][(size_t)y * Ly];
                        for (int ky = 0; ky < Ly; ++ky) dst[ky] += s1 * row[ky];
                    }
                }
            // stage z: out[kx][ky][kz] = sign scale sum_z S2[z][kx][ky] row_z[z][kz]
            double *out = spec.data() + (size_t)c * H * Ly * Lz;
            for (int kx = 0; kx < H; ++kx)
                for (int ky = 0; ky < Ly; ++ky) {
                    double *dst = out + ((size_t)kx * Ly + ky) * Lz;
                    for (int z = 0; z < Bz; ++z) {
                        const double s2 = S2[((size_t)z * H + kx) * Ly + ky];
                        const double *row = &rz[oddz][(size_t)z * Lz];
                        for (int kz = 0; kz < Lz; ++kz) dst[kz] += s2 * row[kz];
                    }
                    for (int kz = 0; kz < Lz; ++kz) dst[kz] *= sign * scale;
                }
        }
}

// D^e table (eq. (mat:se)): for a node whose clamped distances (in nodes, capped at
// M) to the low/high faces of each axis are (lo_a, hi_a), the sum of the bond
// weights of the offsets that leave the grid.  Index: digits (lo_x, hi_x, lo_y,
// hi_y[, lo_z, hi_z]) in base M+1, first digit most significant.
static void build_de_table(const msb_plan_s *p, const std::vector<long double> &W,
                           std::vector<double> &de) {
    const int d = p->dim, M = p->M, nc = p->ncomp, nd = 2 * d;
    const int S = p->de_stride;
    de.assign((size_t)nc * S, 0.0);
    std::vector<int> dig(nd);
    for (int idx = 0; idx < S; ++idx) {
        int t = idx;
        for (int q = nd - 1; q >= 0; --q) {
            dig[q] = t % (M + 1);
            t /= (M + 1);
        }
        std::vector<long double> acc(nc, 0.0L);
        for (int i = 0; i < p->n_off; ++i) {
            const int *o = &p->off[3 * i];
            bool out = false;
            for (int a = 0; a < d; ++a)
                if (o[a] < -dig[2 * a] || o[a] > dig[2 * a + 1]) out = true;
            if (!out) continue;
            for (int c = 0; c < nc; ++c) acc[c] += W[(size_t)c * p->n_off + i];
        }
        for (int c = 0; c < nc; ++c) de[(size_t)c * S + idx] = (double)acc[c];
    }
}

// Spectra of the generating array wrapped to a tl x tl frame (the tiled 2D product):
// Ghat(k) = sum_o K(o) exp(-2 pi i k.o / tl) over the (2M+1)^2 box; K is even in o for
// every component, so the sum is real, sum_o K(o) cos(2 pi k.o / tl), each cosine taken
// from the exact unit circle at (k.o mod tl).  Stored as the three reals the product
// uses per frequency, (Gxx + Gyy)/2, (Gxx - Gyy)/2 and Gxy, scaled by 1/tl^2 (the
// inverse transform's factor): out[c][ky][kx].
static void tile_spectrum(const msb_plan_s *p, const std::vector<long double> &W, int tl, std::vector<double> &out) {
    std::vector<long double> cs, sn;
    unit_circle(tl, cs, sn);
    const int n2 = tl * tl;
    std::vector<long double> g((size_t)3 * n2, 0.0L);
    long double centre[3] = {0.0L, 0.0L, 0.0L};
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < p->n_off; ++i) centre[c] -= W[(size_t)c * p->n_off + i];   // eq. (frb:e4)
    for (int ky = 0; ky < tl; ++ky)
        for (int kx = 0; kx < tl; ++kx) {
            long double acc[3] = {centre[0], centre[1], centre[2]};
            for (int i = 0; i < p->n_off; ++i) {
                const int *o = &p->off[3 * i];
                long long t = ((long long)kx * o[0] + (long long)ky * o[1]) % tl;
                if (t < 0) t += tl;
                const long double cv = cs[t];
                for (int c = 0; c < 3; ++c) acc[c] += W[(size_t)c * p->n_off + i] * cv;
            }
            const size_t k = (size_t)ky * tl + kx;
            g[k] = acc[0];
            g[n2 + k] = acc[1];
            g[2 * (size_t)n2 + k] = acc[2];
        }
    const long double sc = 1.0L / ((long double)tl * tl);
    out.assign((size_t)3 * n2, 0.0);
    for (int k = 0; k < n2; ++k) {
        const long double gxx = g[k], gxy = g[n2 + k], gyy = g[2 * (size_t)n2 + k];
        out[k] = (double)(0.5L * (gxx + gyy) * sc);
        out[n2 + k] = (double)(0.5L * (gxx - gyy) * sc);
        out[2 * (size_t)n2 + k] = (double)(gxy * sc);
    }
}

template <typename T> static msb_status upload(T **dst, const std::vector<T> &v) {
    if (*dst) { hipFree(*dst); *dst = nullptr; }
    if (v.empty()) return MSB_OK;
    MSB_HIP(hipMalloc(dst, sizeof(T) * v.size()));
    MSB_HIP(hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return MSB_OK;
}

size_t de_len(const msb_plan_s *p) { return (size_t)p->ncomp * p->de_stride; }
size_t w_len(const msb_plan_s *p) { return (size_t)p->ncomp * p->n_off; }

msb_status alloc_operator(msb_plan_s *p, DeviceOp &op, int count) {
    free_operator(op);
    const size_t ns = (size_t)p->ncomp * spectrum_len(p) * count;
    const size_t nd = de_len(p) * count, nw = w_len(p) * count;
    op.count = count;
    MSB_HIP(hipMalloc(&op.spec64, sizeof(double) * ns));
    MSB_HIP(hipMalloc(&op.spec32, sizeof(float) * ns));
    MSB_HIP(hipMalloc(&op.de64, sizeof(double) * nd));
    MSB_HIP(hipMalloc(&op.de32, sizeof(float) * nd));
    MSB_HIP(hipMalloc(&op.w64, sizeof(double) * nw));
    MSB_HIP(hipMalloc(&op.w32, sizeof(float) * nw));
    return MSB_OK;
}

template <typename T> static msb_status put(T *dst, const std::vector<double> &v) {
    std::vector<T> t(v.begin(), v.end());
    MSB_HIP(hipMemcpy(dst, t.data(), sizeof(T) * t.size(), hipMemcpyHostToDevice));
    return MSB_OK;
}

// Coefficients of operator slot c (shared, or case c's with per-case coefficients).
static std::vector<double> slot_infl(const msb_plan_s *p, int c) {
    if (!p->per_case) return p->infl;
    return std::vector<double>(p->infl_case.begin() + (size_t)c * p->n_infl,
                               p->infl_case.begin() + (size_t)(c + 1) * p->n_infl);
}

// Circulant preconditioner of K = -A: on the padded grid, the periodic operator with
// the same generating array is diagonal in Fourier space with the d x d real symmetric
// blocks Khat(k) = -Ghat(k).  Its shifted inverse (Khat(k) + s I)^{-1}, s = 1e-3 times
// the largest block eigenvalue bound (which also removes the rigid-motion nullspace at
// k = 0), is stored like the spectra (components xx xy yy / xx xy xz yy yz zz, scaled
// by 1 / prod(L)), so the same product chain applies it.
// Host part of one slot of the preconditioner (reads only the plan's geometry: several
// plans may run it on parallel threads).
static void precond_symbol(const msb_plan_s *p, const std::vector<double> &infl, std::vector<double> &out) {
    const int d = p->dim, nc = p->ncomp;
    const size_t ns = spectrum_len(p);
    const double vol = (double)p->L[0] * (double)p->L[1] * (double)p->L[2];
    std::vector<long double> W;
    bond_weights(p, infl, W);
    std::vector<double> spec;
    build_spectrum(p, W, spec);
    out.assign((size_t)nc * ns, 0.0);
    // Khat = -spec * vol per frequency; largest eigenvalue bound by the row sums
    double lmax = 0.0;
    for (size_t k = 0; k < ns; ++k) {
        double Kb[3][3];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) Kb[a][b] = -spec[(size_t)comp_index(a, b, d) * ns + k] * vol;
        for (int a = 0; a < d; ++a) {
            double r = 0.0;
            for (int b = 0; b < d; ++b) r += std::fabs(Kb[a][b]);
            lmax = std::max(lmax, r);
        }
    }
    const double shift = 1e-3 * (lmax > 0.0 ? lmax : 1.0);
    for (size_t k = 0; k < ns; ++k) {
        double Kb[3][3], I[3][3];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) Kb[a][b] = -spec[(size_t)comp_index(a, b, d) * ns + k] * vol + (a == b ? shift : 0.0);
        if (d == 2) {
            const double det = Kb[0][0] * Kb[1][1] - Kb[0][1] * Kb[1][0];
            I[0][0] = Kb[1][1] / det;
            I[1][1] = Kb[0][0] / det;
            I[0][1] = I[1][0] = -Kb[0][1] / det;
        } else {
            const double c00 = Kb[1][1] * Kb[2][2] - Kb[1][2] * Kb[2][1];
            const double c01 = Kb[1][2] * Kb[2][0] - Kb[1][0] * Kb[2][2];
            const double c02 = Kb[1][0] * Kb[2][1] - Kb[1][1] * Kb[2][0];
            const double det = Kb[0][0] * c00 + Kb[0][1] * c01 + Kb[0][2] * c02;
            I[0][0] = c00 / det;
            I[0][1] = I[1][0] = c01 / det;
            I[0][2] = I[2][0] = c02 / det;
            I[1][1] = (Kb[0][0] * Kb[2][2] - Kb[0][2] * Kb[2][0]) / det;
            I[1][2] = I[2][1] = (Kb[0][2] * Kb[1][0] - Kb[0][0] * Kb[1][2]) / det;
            I[2][2] = (Kb[0][0] * Kb[1][1] - Kb[0][1] * Kb[1][0]) / det;
        }
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b) out[(size_t)comp_index(a, b, d) * ns + k] = I[a][b] / vol;
    }
}

// Runs body(i) for i in [0, n) on up to 16 host threads (the plans' host preparation
// work; each i touches only its own outputs).  Returns false if a thread failed.
static bool parallel_for(int n, const std::function<void(int)> &body) {
    const int nt = std::max(1, std::min({n, 16, (int)std::max(1u, std::thread::hardware_concurrency())}));
    std::atomic<int> next{0};
    std::atomic<bool> ok{true};
    auto work = [&]() {
        for (int i = next++; i < n; i = next++) {
            try {
                body(i);
            } catch (...) {
                ok = false;
            }
        }
    };
    if (nt <= 1) {
        work();
        return ok;
    }
    std::vector<std::thread> th;
    try {
        for (int t = 1; t < nt; ++t) th.emplace_back(work);
    } catch (...) {   // fewer threads than asked: the remaining ones share the work
    }
    work();
    for (auto &t : th) t.join();
    return ok;
}

// Preconditioners of every listed plan that has none: the symbols on parallel host
// threads, then the uploads in plan order.
msb_status build_preconditioners(msb_plan_s *const *ps, int n) {
    std::vector<int> todo;
    for (int i = 0; i < n; ++i)
        if (ps[i]->pre.count <= 0) todo.push_back(i);
    std::vector<std::vector<std::vector<double>>> sym(todo.size());
    const bool ok = parallel_for((int)todo.size(), [&](int k) {
        const msb_plan_s *p = ps[todo[k]];
        const int count = p->op.count > 0 ? p->op.count : 1;
        sym[k].resize(count);
        for (int c = 0; c < count; ++c) precond_symbol(p, slot_infl(p, c), sym[k][c]);
    });
    MSB_CHECK(ok, MSB_ENOMEM, "host allocation failed while building preconditioners");
    for (size_t k = 0; k < todo.size(); ++k) {
        msb_plan_s *p = ps[todo[k]];
        DeviceOp &pre = p->pre;
        const int count = (int)sym[k].size();
        const size_t all = (size_t)p->ncomp * spectrum_len(p);
        free_operator(pre);
        MSB_HIP(hipMalloc(&pre.spec64, sizeof(double) * all * count));
        MSB_HIP(hipMalloc(&pre.spec32, sizeof(float) * all * count));
        for (int c = 0; c < count; ++c) {
            MSB_TRY(put(pre.spec64 + all * c, sym[k][c]));
            MSB_TRY(put(pre.spec32 + all * c, sym[k][c]));
        }
        pre.count = count;   // built (a failed build leaves count 0: rebuilt on next use)
    }
    return MSB_OK;
}

msb_status build_preconditioner(msb_plan_s *p) {
    free_operator(p->pre);
    return build_preconditioners(&p, 1);
}

// Fictitious density of the dynamic-relaxation solver (the cited ADR method): a Gershgorin
// bound per row, D_ii = 1/4 sum_j |K_ij| with K = -A as the products apply it (in-grid
// neighbours, broken bonds removed, surface factors on Omega_e rows): off-diagonal blocks
// |W(o)| per neighbour, the diagonal block |sum_o W(o)|.
void build_adr_density(const msb_plan_s *p, std::vector<double> &D, int &slots) {
    const int d = p->dim, M = p->M;
    slots = p->op.count > 1 ? p->op.count : 1;
    const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2], N = p->N;
    // broken neighbours per node (CSR from the sorted pair list)
    std::vector<int64_t> ptr(N + 1, 0), nb;
    const int64_t np_ = p->n_pairs;
    for (int64_t e = 0; e < np_; ++e) {
        ptr[p->bonds_host[2 * e] + 1]++;
        ptr[p->bonds_host[2 * e + 1] + 1]++;
    }
    for (int64_t i = 0; i < N; ++i) ptr[i + 1] += ptr[i];
    nb.assign(ptr[N], 0);
    {
        std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t e = 0; e < np_; ++e) {
            const int64_t a = p->bonds_host[2 * e], b = p->bonds_host[2 * e + 1];
            nb[fill[a]++] = b;
            nb[fill[b]++] = a;
        }
    }
    const bool surf = !p->nu_host.empty();
    D.assign((size_t)slots * d * N, 0.0);
    for (int sl = 0; sl < slots; ++sl) {
        const std::vector<double> infl = p->per_case ? std::vector<double>(p->infl_case.begin() + (size_t)sl * p->n_infl,
                                                                           p->infl_case.begin() + (size_t)(sl + 1) * p->n_infl)
                                                     : p->infl;
        std::vector<long double> Wl;
        bond_weights(p, infl, Wl);
        std::vector<double> W(Wl.begin(), Wl.end());   // [comp][n_off]
        double *Ds = D.data() + (size_t)sl * d * N;
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t pn = (k * ny + j) * nx + i;
                    const bool on_e = surf && (i < M || i >= nx - M || j < M || j >= ny - M ||
                                               (d == 3 && (k < M || k >= nz - M)));
                    double off[3] = {0, 0, 0}, diag[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                    for (int o = 0; o < p->n_off; ++o) {
                        const int *of = &p->off[3 * o];
                        const int64_t x = i + of[0], y = j + of[1], z = k + of[2];
                        if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) continue;
                        const int64_t q = (z * ny + y) * nx + x;
                        bool broken = false;
                        for (int64_t t = ptr[pn]; t < ptr[pn + 1] && !broken; ++t) broken = nb[t] == q;
                        if (broken) continue;
                        const double v = on_e ? 0.5 * (p->nu_host[pn] + p->nu_host[q]) : 1.0;
                        for (int a = 0; a < d; ++a)
                            for (int c = 0; c < d; ++c) {
                                const double wv = v * W[(size_t)comp_index(a, c, d) * p->n_off + o];
                                off[a] += std::fabs(wv);
                                diag[a][c] += wv;
                            }
                    }
                    for (int a = 0; a < d; ++a) {
                        double r = off[a];
                        for (int c = 0; c < d; ++c) r += std::fabs(diag[a][c]);
                        Ds[(size_t)a * N + pn] = 0.25 * r;
                    }
                }
    }
}

// Fill one slot of an operator for the given influence coefficients.
// Host part of one operator slot: spectra, D^e table and bond weights (reads only the
// plan's geometry: several plans may run it on parallel threads).
struct OperatorHost {
    std::vector<double> spec, de, w;
};
static void operator_host(const msb_plan_s *p, const std::vector<double> &infl, OperatorHost &h) {
    std::vector<long double> W;
    bond_weights(p, infl, W);
    build_spectrum(p, W, h.spec);
    build_de_table(p, W, h.de);
    h.w.assign(W.begin(), W.end());
}

static void free_tiles(DeviceOp &op) {
    for (TileSpec &t : op.tiles) {
        if (t.s64) (void)hipFree(t.s64);
        if (t.s32) (void)hipFree(t.s32);
        if (t.r64) (void)hipFree(t.r64);
        if (t.r32) (void)hipFree(t.r32);
    }
    op.tiles.clear();
}

static msb_status upload_operator(msb_plan_s *p, const OperatorHost &h, DeviceOp &op, int slot,
                                  const std::vector<double> &infl) {
    const size_t ns = (size_t)p->ncomp * spectrum_len(p), nd = de_len(p), nw = w_len(p);
    free_tiles(op);   // frame spectra of the old coefficients (rebuilt by ensure_tiles)
    if ((int)op.infl_slots.size() < op.count) op.infl_slots.resize(op.count);
    op.infl_slots[slot] = infl;
    MSB_TRY(put(op.spec64 + ns * slot, h.spec));
    MSB_TRY(put(op.spec32 + ns * slot, h.spec));
    MSB_TRY(put(op.de64 + nd * slot, h.de));
    MSB_TRY(put(op.de32 + nd * slot, h.de));
    MSB_TRY(put(op.w64 + nw * slot, h.w));
    MSB_TRY(put(op.w32 + nw * slot, h.w));
    return MSB_OK;
}

msb_status fill_operator(msb_plan_s *p, const std::vector<double> &infl, DeviceOp &op, int slot) {
    OperatorHost h;
    operator_host(p, infl, h);
    return upload_operator(p, h, op, slot, infl);
}

void free_operator(DeviceOp &op) {
    void *b[] = {op.spec64, op.spec32, op.de64, op.de32, op.w64, op.w32};
    for (void *x : b)
        if (x) hipFree(x);
    free_tiles(op);
    op = DeviceOp();
}

const TileSpec *find_tile_spec(const DeviceOp &op, int tl) {
    for (const TileSpec &t : op.tiles)
        if (t.tl == tl) return &t;
    return nullptr;
}

const FftAxis *find_tile_axis(const msb_plan_s *p, int tl) {
    for (const FftAxis &a : p->tax)
        if (a.L == tl) return &a;
    return nullptr;
}

// Frame spectra of one operator for length tl (all its slots, both precisions).
static msb_status build_tile_spec(msb_plan_s *p, DeviceOp &op, int tl) {
    const size_t n = (size_t)3 * tl * tl;
    std::vector<double> all(n * op.count);
    for (int c = 0; c < op.count; ++c) {
        std::vector<long double> W;
        bond_weights(p, c < (int)op.infl_slots.size() ? op.infl_slots[c] : p->infl, W);
        std::vector<double> v;
        tile_spectrum(p, W, tl, v);
        std::copy(v.begin(), v.end(), all.begin() + n * c);
    }
    TileSpec t;
    t.tl = tl;
    MSB_TRY(upload(&t.s64, all));
    msb_status st = upload(&t.s32, std::vector<float>(all.begin(), all.end()));
    // the register-frame order: R points per thread at kx = p + S i of line ky = ln, thread
    // t = p tl + ln; entry (i, t) of each component block
    const int R = tl == 16 ? 4 : 8, S = tl == 64 ? 8 : 4;
    if (st == MSB_OK && (tl == 16 || tl == 32 || tl == 64)) {
        std::vector<double> reg(all.size());
        const size_t blk = (size_t)tl * tl;
        for (size_t k = 0; k < (size_t)3 * op.count; ++k)
            for (int i = 0; i < R; ++i)
                for (int th = 0; th < S * tl; ++th) {
                    const int ky = th % tl, kx = th / tl + S * i;
                    reg[k * blk + (size_t)i * S * tl + th] = all[k * blk + (size_t)ky * tl + kx];
                }
        st = upload(&t.r64, reg);
        if (st == MSB_OK) st = upload(&t.r32, std::vector<float>(reg.begin(), reg.end()));
    }
    if (st != MSB_OK) {
        for (void *x : {(void *)t.s64, (void *)t.s32, (void *)t.r64, (void *)t.r32})
            if (x) (void)hipFree(x);
        return st;
    }
    op.tiles.push_back(t);
    return MSB_OK;
}

msb_status ensure_tiles(msb_plan_s *p, int extra, bool extra_op_only) {
    if (p->dim != 2) return MSB_OK;
    const int want[3] = {p->cfg[0].tile, p->cfg[1].tile, extra};
    for (int w = 0; w < 3; ++w) {
        const int tl = want[w];
        if (tl <= 0) continue;
        if (!find_tile_axis(p, tl)) {
            FftAxis ax;
            MSB_TRY(make_axis(tl, ax));
            p->tax.push_back(ax);
        }
        if (p->op.count > 0 && !find_tile_spec(p->op, tl)) MSB_TRY(build_tile_spec(p, p->op, tl));
        if (w == 2 && extra_op_only) continue;
        for (DeviceOp &d : p->dop)
            if (d.count > 0 && !find_tile_spec(d, tl)) MSB_TRY(build_tile_spec(p, d, tl));
    }
    return MSB_OK;
}

static msb_status validate_desc(const msb_problem_desc *d) {
    MSB_CHECK(d, MSB_EINVAL, "null problem description");
    MSB_CHECK(d->dim == 2 || d->dim == 3, MSB_EINVAL, "dim must be 2 or 3 (got %d)", d->dim);
    for (int a = 0; a < d->dim; ++a)
        MSB_CHECK(d->n[a] >= 1 && d->n[a] <= (1 << 20), MSB_EINVAL, "n[%d] = %lld out of range", a,
                  (long long)d->n[a]);
    MSB_CHECK(std::isfinite(d->h) && d->h > 0, MSB_EINVAL, "h must be finite and > 0");
    MSB_CHECK(d->M >= 1 && d->M <= 32, MSB_EINVAL, "M must be in [1, 32] (got %d)", d->M);
    MSB_CHECK(d->dim == 2 || d->M <= 10, MSB_EUNSUPPORTED, "3D supports M <= 10 (got %d)", d->M);
    MSB_CHECK(std::isfinite(d->alpha), MSB_EINVAL, "alpha must be finite");
    MSB_CHECK(d->n_infl >= 0 && d->n_infl <= 8, MSB_EINVAL, "n_infl must be in [0, 8]");
    MSB_CHECK(d->n_infl == 0 || d->infl, MSB_EINVAL, "infl is null but n_infl > 0");
    for (int k = 0; k < d->n_infl; ++k)
        MSB_CHECK(std::isfinite(d->infl[k]), MSB_EINVAL, "infl[%d] not finite", k);
    MSB_CHECK(std::isfinite(d->rho) && d->rho > 0, MSB_EINVAL, "rho must be finite and > 0");
    MSB_CHECK(d->batch >= 1 && d->batch <= 4096, MSB_EINVAL, "batch must be in [1, 4096]");
    int64_t N = d->n[0] * d->n[1] * (d->dim == 3 ? d->n[2] : 1);
    MSB_CHECK(N * d->dim * (int64_t)d->batch < (int64_t(1) << 31), MSB_EUNSUPPORTED,
              "B*d*N must stay below 2^31");
    return MSB_OK;
}

}  // namespace msb

using namespace msb;

extern "C" const char *msb_last_error(void) { return g_err.c_str(); }

// Transform workspace: T1 holds the x half spectra [B][d][Nz][H][Ny], T2 (3D) the
// y spectra [B][d][H][Ly][Nz]; sized for complex FP64 and shared by FP32.
static msb_status alloc_transform_ws(msb_plan_s *p) {
    const int d = p->dim;
    const size_t c16 = sizeof(double2);
    p->T1_bytes = (size_t)p->B * d * p->n[2] * p->H * p->n[1] * c16;
    MSB_HIP(hipMalloc(&p->T1, p->T1_bytes));
    if (d == 3) {
        p->T2_bytes = (size_t)p->B * d * p->H * p->L[1] * p->n[2] * c16;
        MSB_HIP(hipMalloc(&p->T2, p->T2_bytes));
    }
    return MSB_OK;
}

static void free_axes(msb_plan_s *p) {
    for (int a = 0; a < 3; ++a) {
        if (p->ax[a].tw64) (void)hipFree(p->ax[a].tw64);
        if (p->ax[a].tw32) (void)hipFree(p->ax[a].tw32);
        p->ax[a] = FftAxis();
    }
    for (FftAxis &t : p->tax) {
        if (t.tw64) (void)hipFree(t.tw64);
        if (t.tw32) (void)hipFree(t.tw32);
    }
    p->tax.clear();
}

// Largest padded length per axis: the x pass stages up to three length-L signals
// in LDS and the Stockham index split (fdiv) is exact while signals * (L/R)^2 < 2^32.
constexpr int64_t kMaxLength = 16384;

static msb_status check_lengths(const msb_plan_s *p, const int64_t *L) {
    for (int a = 0; a < p->dim; ++a) {
        MSB_CHECK(L[a] >= p->n[a] + p->M, MSB_EINVAL, "L[%d] = %lld < N + M = %lld", a, (long long)L[a],
                  (long long)(p->n[a] + p->M));
        MSB_CHECK(L[a] <= kMaxLength, MSB_EUNSUPPORTED, "L[%d] = %lld exceeds %lld", a, (long long)L[a],
                  (long long)kMaxLength);
        std::vector<int> r;
        MSB_CHECK(factor_length((int)L[a], r, 16), MSB_EINVAL, "L[%d] = %lld has a prime factor above 5", a,
                  (long long)L[a]);
    }
    return MSB_OK;
}

// Build the parts of the plan that depend on the padded lengths (p->L set).
static msb_status build_layout(msb_plan_s *p) {
    ++p->layout_version;
    p->H = p->L[0] / 2 + 1;
    for (int a = 0; a < 3; ++a) MSB_TRY(make_axis((int)p->L[a], p->ax[a]));
    const int count = p->op.count > 0 ? p->op.count : 1;
    MSB_TRY(alloc_operator(p, p->op, count));
    for (int c = 0; c < count; ++c) {
        std::vector<double> v = p->per_case ? std::vector<double>(p->infl_case.begin() + (size_t)c * p->n_infl,
                                                                  p->infl_case.begin() + (size_t)(c + 1) * p->n_infl)
                                            : p->infl;
        MSB_TRY(fill_operator(p, v, p->op, c));
    }
    for (auto &o : p->dop) free_operator(o);
    p->dop.clear();
    free_operator(p->pre);
    MSB_TRY(alloc_transform_ws(p));
    for (int f = 0; f < 2; ++f) {
        p->cfg[f] = default_config(p, f == 1);
        MSB_TRY(set_schedules(p, f == 1, p->cfg[f].max_radix));
        MSB_CHECK(check_config(p, f == 1, p->cfg[f]) == MSB_OK, MSB_EUNSUPPORTED,
                  "grid too large for the LDS-staged transforms (%s)", msb_last_error());
    }
    return ensure_tiles(p);
}

msb_status msb::relayout(msb_plan_s *p, const int64_t *L) {
    int64_t Ln[3] = {1, 1, 1};
    for (int a = 0; a < p->dim; ++a) Ln[a] = L[a];
    MSB_TRY(check_lengths(p, Ln));
    MSB_HIP(hipDeviceSynchronize());
    free_axes(p);
    if (p->T1) (void)hipFree(p->T1);
    if (p->T2) (void)hipFree(p->T2);
    p->T1 = p->T2 = nullptr;
    for (int a = 0; a < 3; ++a) p->L[a] = Ln[a];
    return build_layout(p);
}

extern "C" msb_status msb_plan_create(const msb_problem_desc *desc, msb_plan *out) {
    MSB_CHECK(out, MSB_EINVAL, "null output pointer");
    *out = nullptr;
    MSB_TRY(validate_desc(desc));
    msb_plan_s *p = new (std::nothrow) msb_plan_s();
    MSB_CHECK(p, MSB_ENOMEM, "host allocation failed");
    hipGetDevice(&p->device);
    p->dim = desc->dim;
    p->n[0] = desc->n[0];
    p->n[1] = desc->n[1];
    p->n[2] = desc->dim == 3 ? desc->n[2] : 1;
    p->N = p->n[0] * p->n[1] * p->n[2];
    p->h = desc->h;
    p->M = desc->M;
    p->alpha = desc->alpha;
    p->n_infl = desc->n_infl;
    p->infl.assign(desc->infl, desc->infl + desc->n_infl);
    p->rho = desc->rho;
    p->B = desc->batch;
    p->ncomp = desc->dim == 2 ? 3 : 6;

    // padded lengths: any L >= N + M gives the exact linear product (support +-M)
    for (int a = 0; a < 3; ++a) p->L[a] = a < p->dim ? next_smooth((int)(p->n[a] + p->M), false) : 1;
    p->de_stride = 1;
    for (int q = 0; q < 2 * p->dim; ++q) p->de_stride *= (p->M + 1);
    build_offsets(p);
    msb_status st = check_lengths(p, p->L);
    if (st == MSB_OK) st = upload(&p->off_dev, std::vector<int32_t>(p->off.begin(), p->off.end()));
    if (st == MSB_OK) st = build_layout(p);
    if (st != MSB_OK) {
        msb_plan_destroy(p);
        return st;
    }
    *out = p;
    return MSB_OK;
}

extern "C" void msb_plan_destroy(msb_plan p) {
    if (!p) return;
    hipDeviceSynchronize();
    free_axes(p);
    free_operator(p->op);
    free_operator(p->pre);
    for (auto &o : p->dop) free_operator(o);
    void *bufs[] = {p->fixed, p->row_fix, p->fix_sat, p->br_row_ptr, p->br_node_i, p->br_bond_ptr, p->br_q, p->br_off, p->T1, p->T2,
                    p->nu64, p->nu32, p->off_dev};
    for (void *b : bufs)
        if (b) hipFree(b);
    solver_cache_free(p);
    crack_free(p);
    delete p;
}

extern "C" msb_status msb_plan_info(msb_plan p, int64_t *L, int64_t *N, int64_t *n_bonds) {
    MSB_CHECK(p, MSB_EINVAL, "null plan");
    if (L)
        for (int a = 0; a < 3; ++a) L[a] = p->L[a];
    if (N) *N = p->N;
    if (n_bonds) *n_bonds = p->n_pairs;
    return MSB_OK;
}

extern "C" msb_status msb_plan_set_constraints(msb_plan p, const uint8_t *fixed) {
    MSB_CHECK(p, MSB_EINVAL, "null plan");
    ++p->op_version;
    const size_t n = (size_t)p->dim * p->N;
    if (!fixed) {
        if (p->fixed) hipFree(p->fixed);
        if (p->row_fix) hipFree(p->row_fix);
        if (p->fix_sat) hipFree(p->fix_sat);
        p->fixed = nullptr;
        p->row_fix = nullptr;
        p->fix_sat = nullptr;
        p->n_fixed = 0;
        return MSB_OK;
    }
    std::vector<uint8_t> v(fixed, fixed + n);
    int64_t cnt = 0;
    for (auto &x : v) {
        x = x ? 1 : 0;
        cnt += x;
    }
    // the class of every x-row of every component (no constrained DOF / all / some), so that
    // the x-inverse reads the mask only on rows with some
    const int64_t nx = p->n[0], rows = p->N / nx;
    std::vector<uint8_t> rc((size_t)p->dim * rows);
    for (int64_t r = 0; r < (int64_t)rc.size(); ++r) {
        int64_t k = 0;
        for (int64_t i = 0; i < nx; ++i) k += v[(size_t)r * nx + i];
        rc[r] = k == 0 ? 0 : (k == nx ? 1 : 2);
    }
    if (!p->fixed) MSB_HIP(hipMalloc(&p->fixed, n));
    if (!p->row_fix) MSB_HIP(hipMalloc(&p->row_fix, rc.size()));
    MSB_HIP(hipMemcpy(p->fixed, v.data(), n, hipMemcpyHostToDevice));
    MSB_HIP(hipMemcpy(p->row_fix, rc.data(), rc.size(), hipMemcpyHostToDevice));
    if (p->dim == 2) {
        // summed-area table of the constrained DOFs (both components) for the tiled product:
        // a block whose inner nodes hold none reads no mask
        const int64_t ny = p->n[1], W = nx + 1;
        std::vector<int32_t> sat((size_t)(ny + 1) * W, 0);
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int32_t k = v[(size_t)y * nx + x] + v[(size_t)p->N + y * nx + x];
                sat[(size_t)(y + 1) * W + x + 1] = sat[(size_t)y * W + x + 1] + sat[(size_t)(y + 1) * W + x] -
                                                   sat[(size_t)y * W + x] + k;
            }
        if (!p->fix_sat) MSB_HIP(hipMalloc(&p->fix_sat, sizeof(int32_t) * sat.size()));
        MSB_HIP(hipMemcpy(p->fix_sat, sat.data(), sizeof(int32_t) * sat.size(), hipMemcpyHostToDevice));
    }
    p->n_fixed = cnt;
    return MSB_OK;
}

extern "C" msb_status msb_plan_set_bonds(msb_plan p, const int64_t *pairs, int64_t nb) {
    MSB_CHECK(p, MSB_EINVAL, "null plan");
    MSB_TRY(msb::set_bonds_impl(p, pairs, nb));
    p->mu_valid = false;
    return MSB_OK;
}

extern "C" msb_status msb_plan_set_surface(msb_plan p, const double *nu) {
    MSB_CHECK(p, MSB_EINVAL, "null plan");
    ++p->op_version;
    if (!nu) {
        if (p->nu64) hipFree(p->nu64);
        if (p->nu32) hipFree(p->nu32);
        p->nu64 = nullptr;
        p->nu32 = nullptr;
        p->nu_host.clear();
        return MSB_OK;
    }
    std::vector<double> v(nu, nu + p->N);
    for (int64_t i = 0; i < p->N; ++i)
        MSB_CHECK(std::isfinite(v[i]) && v[i] > 0.0, MSB_EINVAL, "surface factor %lld must be finite and > 0",
                  (long long)i);
    MSB_TRY(upload(&p->nu64, v));
    MSB_TRY(upload(&p->nu32, std::vector<float>(v.begin(), v.end())));
    p->nu_host = v;
    return MSB_OK;
}

extern "C" msb_status msb_surface_volume_factors(msb_plan p, double *nu) {
    MSB_CHECK(p && nu, MSB_EINVAL, "null argument");
    const int d = p->dim, M = p->M;
    std::vector<double> lam(p->n_off);
    double full = 0.0;
    for (int i = 0; i < p->n_off; ++i) {
        const int *o = &p->off[3 * i];
        const long long s2 = (long long)o[0] * o[0] + (long long)o[1] * o[1] + (long long)o[2] * o[2];
        lam[i] = s2 <= (long long)M * M - M ? 1.0 : M + 0.5 - std::sqrt((double)s2);
        full += lam[i];
    }
    const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const bool inner = i >= M && i < nx - M && j >= M && j < ny - M && (d == 2 || (k >= M && k < nz - M));
                double in = full;
                if (!inner) {
                    in = 0.0;
                    for (int t = 0; t < p->n_off; ++t) {
                        const int *o = &p->off[3 * t];
                        const int64_t x = i + o[0], y = j + o[1], z = k + o[2];
                        if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) in += lam[t];
                    }
                }
                nu[(k * ny + j) * nx + i] = full / in;
            }
    return MSB_OK;
}

extern "C" msb_status msb_plan_get_bonds(msb_plan p, int64_t *pairs, int64_t cap, int64_t *count) {
    MSB_CHECK(p, MSB_EINVAL, "null plan");
    MSB_CHECK(count, MSB_EINVAL, "null count");
    *count = p->n_pairs;
    MSB_CHECK(cap >= 0, MSB_EINVAL, "negative capacity");
    if (pairs && cap > 0) {
        const int64_t n = std::min<int64_t>(cap, p->n_pairs);
        std::memcpy(pairs, p->bonds_host.data(), sizeof(int64_t) * 2 * n);
    }
    return MSB_OK;
}

msb_status msb::set_bonds_impl(msb_plan_s *p, const int64_t *pairs, int64_t nb) {
    MSB_CHECK(nb >= 0, MSB_EINVAL, "negative bond count");
    MSB_CHECK(nb == 0 || pairs, MSB_EINVAL, "null bond list");
    const int d = p->dim, M = p->M, B = 2 * M + 1;
    const int64_t nx = p->n[0], ny = p->n[1];
    // offset -> stencil id lookup
    std::vector<int> lut((size_t)B * B * B, -1);
    for (int i = 0; i < p->n_off; ++i) {
        const int *o = &p->off[3 * i];
        lut[((size_t)(o[2] + M) * B + (o[1] + M)) * B + (o[0] + M)] = i;
    }
    struct Dir { int64_t p, q; int off; };
    std::vector<Dir> dir;
    dir.reserve(2 * nb);
    for (int64_t e = 0; e < nb; ++e) {
        int64_t a = pairs[2 * e], b = pairs[2 * e + 1];
        MSB_CHECK(a >= 0 && a < p->N && b >= 0 && b < p->N && a != b, MSB_EINVAL,
                  "bond %lld: node ids (%lld, %lld) invalid", (long long)e, (long long)a, (long long)b);
        int64_t ia[3] = {a % nx, (a / nx) % ny, a / (nx * ny)};
        int64_t ib[3] = {b % nx, (b / nx) % ny, b / (nx * ny)};
        int o[3] = {0, 0, 0};
        int64_t s2 = 0;
        for (int c = 0; c < d; ++c) {
            int64_t t = ib[c] - ia[c];
            MSB_CHECK(t >= -M && t <= M, MSB_EINVAL, "bond %lld outside the horizon", (long long)e);
            o[c] = (int)t;
            s2 += t * t;
        }
        MSB_CHECK(s2 <= (int64_t)M * M, MSB_EINVAL, "bond %lld outside the horizon", (long long)e);
        int id = lut[((size_t)(o[2] + M) * B + (o[1] + M)) * B + (o[0] + M)];
        int idn = lut[((size_t)(-o[2] + M) * B + (-o[1] + M)) * B + (-o[0] + M)];
        dir.push_back({a, b, id});
        dir.push_back({b, a, idn});
    }
    std::sort(dir.begin(), dir.end(), [](const Dir &x, const Dir &y) {
        return x.p != y.p ? x.p < y.p : x.q < y.q;
    });
    for (size_t i = 1; i < dir.size(); ++i)
        MSB_CHECK(!(dir[i].p == dir[i - 1].p && dir[i].q == dir[i - 1].q), MSB_EINVAL,
                  "duplicate bond (%lld, %lld)", (long long)dir[i].p, (long long)dir[i].q);

    const int64_t rows = rows_total(p);
    std::vector<int32_t> row_ptr(rows + 1, 0), node_i, bond_ptr, q, off;
    for (size_t i = 0; i < dir.size();) {
        size_t j = i;
        while (j < dir.size() && dir[j].p == dir[i].p) ++j;
        int64_t node = dir[i].p;
        row_ptr[node / nx + 1] += 1;
        node_i.push_back((int32_t)node);
        bond_ptr.push_back((int32_t)q.size());
        for (size_t k = i; k < j; ++k) {
            q.push_back((int32_t)dir[k].q);
            off.push_back(dir[k].off);
        }
        i = j;
    }
    bond_ptr.push_back((int32_t)q.size());
    for (int64_t r = 0; r < rows; ++r) row_ptr[r + 1] += row_ptr[r];

    // the five device lists are built first and replace the plan's only when every upload
    // succeeded: a failure leaves the previous broken set complete
    int32_t *nl[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    const std::vector<int32_t> empty;
    const std::vector<int32_t> *src[5] = {nb ? &row_ptr : &empty, &node_i, nb ? &bond_ptr : &empty, &q, &off};
    msb_status us = MSB_OK;
    for (int k = 0; k < 5 && us == MSB_OK; ++k) us = upload(&nl[k], *src[k]);
    if (us != MSB_OK) {
        for (int32_t *b : nl)
            if (b) (void)hipFree(b);
        return us;
    }
    int32_t **cur[5] = {&p->br_row_ptr, &p->br_node_i, &p->br_bond_ptr, &p->br_q, &p->br_off};
    for (int k = 0; k < 5; ++k) {
        if (*cur[k]) (void)hipFree(*cur[k]);
        *cur[k] = nl[k];
    }
    ++p->op_version;
    p->n_pairs = nb;
    p->n_br_nodes = (int64_t)node_i.size();
    std::vector<int64_t> hb;
    hb.reserve(2 * (size_t)nb);
    for (const Dir &e : dir)
        if (e.p < e.q) {
            hb.push_back(e.p);
            hb.push_back(e.q);
        }
    p->bonds_host.swap(hb);   // sorted by (p, q): dir is
    return MSB_OK;
}

// ------------------------------------------------------------------ crack -> bonds
// Orientation of c relative to the directed line a -> b (cross product, FP64).
static inline double orient(double ax, double ay, double bx, double by, double cx, double cy) {
    double u1 = bx - ax, v1 = cy - ay;
    double u2 = by - ay, v2 = cx - ax;
    volatile double t1 = u1 * v1;   // no contraction into an FMA
    volatile double t2 = u2 * v2;
    return t1 - t2;
}

static inline bool strictly_opposite(double s, double t) {
    return (s > 0 && t < 0) || (s < 0 && t > 0);
}

extern "C" msb_status msb_crack_to_bonds(const msb_problem_desc *desc, const double *seg,
                                         int64_t ns, int64_t *pairs_out, int64_t cap,
                                         int64_t *nb_out) {
    MSB_CHECK(desc && nb_out, MSB_EINVAL, "null argument");
    *nb_out = 0;
    MSB_TRY(validate_desc(desc));
    MSB_CHECK(desc->dim == 2, MSB_EUNSUPPORTED, "crack segments are 2D only");
    MSB_CHECK(ns >= 0 && (ns == 0 || seg), MSB_EINVAL, "bad segment list");
    const int64_t nx = desc->n[0], ny = desc->n[1];
    const int M = desc->M;
    const double h = desc->h, delta = M * h;
    std::vector<std::pair<int64_t, int64_t>> out;
    for (int64_t s = 0; s < ns; ++s) {
        const double c0x = seg[4 * s], c0y = seg[4 * s + 1], c1x = seg[4 * s + 2], c1y = seg[4 * s + 3];
        MSB_CHECK(std::isfinite(c0x) && std::isfinite(c0y) && std::isfinite(c1x) && std::isfinite(c1y),
                  MSB_EINVAL, "segment %lld not finite", (long long)s);
        // nodes p that can end a crossing bond lie within delta of the segment's box
        auto lo_idx = [&](double x) {
            double t = std::floor((x - delta) / h - 0.5) - 1;
            return (int64_t)std::max(0.0, t);
        };
        auto hi_idx = [&](double x, int64_t n) {
            double t = std::ceil((x + delta) / h - 0.5) + 1;
            return (int64_t)std::min((double)(n - 1), t);
        };
        int64_t i0 = lo_idx(std::min(c0x, c1x)), i1 = hi_idx(std::max(c0x, c1x), nx);
        int64_t j0 = lo_idx(std::min(c0y, c1y)), j1 = hi_idx(std::max(c0y, c1y), ny);
        for (int64_t j = j0; j <= j1; ++j)
            for (int64_t i = i0; i <= i1; ++i) {
                const double px = (i + 0.5) * h, py = (j + 0.5) * h;
                for (int oy = 0; oy <= M; ++oy)
                    for (int ox = -M; ox <= M; ++ox) {
                        if (oy == 0 && ox <= 0) continue;          // each bond once
                        if (ox * ox + oy * oy > M * M) continue;
                        const int64_t qi = i + ox, qj = j + oy;
                        if (qi < 0 || qi >= nx || qj >= ny) continue;
                        const double qx = (qi + 0.5) * h, qy = (qj + 0.5) * h;
                        double d1 = orient(c0x, c0y, c1x, c1y, px, py);
                        double d2 = orient(c0x, c0y, c1x, c1y, qx, qy);
                        if (!strictly_opposite(d1, d2)) continue;
                        double d3 = orient(px, py, qx, qy, c0x, c0y);
                        double d4 = orient(px, py, qx, qy, c1x, c1y);
                        if (!strictly_opposite(d3, d4)) continue;
                        int64_t a = j * nx + i, b = qj * nx + qi;
                        out.emplace_back(std::min(a, b), std::max(a, b));
                    }
            }
    }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    *nb_out = (int64_t)out.size();
    MSB_CHECK((int64_t)out.size() <= cap, MSB_EINVAL, "bond capacity %lld too small (%lld needed)",
              (long long)cap, (long long)out.size());
    MSB_CHECK(out.empty() || pairs_out, MSB_EINVAL, "null output");
    for (size_t e = 0; e < out.size(); ++e) {
        pairs_out[2 * e] = out[e].first;
        pairs_out[2 * e + 1] = out[e].second;
    }
    return MSB_OK;
}

// New influence coefficients for several plans: validation, the host work of every
// plan on parallel threads, then per plan the uploads and the bookkeeping (derivative
// operators dropped when the coefficient count changes, the preconditioner rebuilt on
// its next use, operator version bumped).  infl[i]: n_infl values, or B_i x n_infl
// with per_case[i] != 0 (per_case may be null).
msb_status msb::set_infl_many(msb_plan_s *const *ps, int n, const double *const *infl, int n_infl,
                              const int *per_case) {
    MSB_CHECK(n_infl >= 0 && n_infl <= 8, MSB_EINVAL, "n_infl must be in [0, 8]");
    for (int i = 0; i < n; ++i) {
        MSB_CHECK(ps[i], MSB_EINVAL, "null plan");
        MSB_CHECK(n_infl == 0 || infl[i], MSB_EINVAL, "null coefficients (plan %d)", i);
        const int64_t nset = (per_case && per_case[i]) ? ps[i]->B : 1;
        for (int64_t k = 0; k < nset * n_infl; ++k)
            MSB_CHECK(std::isfinite(infl[i][k]), MSB_EINVAL, "plan %d: coefficient %lld not finite", i, (long long)k);
    }
    MSB_HIP(hipDeviceSynchronize());
    std::vector<std::vector<OperatorHost>> host(n);
    const bool ok = parallel_for(n, [&](int i) {
        const msb_plan_s *p = ps[i];
        const int count = (per_case && per_case[i]) ? p->B : 1;
        host[i].resize(count);
        for (int c = 0; c < count; ++c) {
            const double *v = n_infl ? infl[i] + (size_t)c * n_infl : nullptr;
            operator_host(p, std::vector<double>(v, v + n_infl), host[i][c]);
        }
    });
    MSB_CHECK(ok, MSB_ENOMEM, "host allocation failed while building the operators");
    for (int i = 0; i < n; ++i) {
        msb_plan_s *p = ps[i];
        ++p->op_version;
        const bool pc = per_case && per_case[i];
        const int count = pc ? p->B : 1;
        if (p->op.count != count) MSB_TRY(alloc_operator(p, p->op, count));
        for (int c = 0; c < count; ++c) {
            const double *v = n_infl ? infl[i] + (size_t)c * n_infl : nullptr;
            MSB_TRY(upload_operator(p, host[i][c], p->op, c, std::vector<double>(v, v + n_infl)));
        }
        p->per_case = pc;
        const double *src = n_infl ? infl[i] : nullptr;
        if (pc) {
            p->infl_case.assign(src, src + (size_t)p->B * n_infl);
            p->infl.clear();
        } else {
            p->infl.assign(src, src + n_infl);
            p->infl_case.clear();
        }
        if (n_infl != p->n_infl) {
            for (auto &o : p->dop) free_operator(o);
            p->dop.clear();
        }
        free_operator(p->pre);   // rebuilt from the new coefficients on the next preconditioned solve
        p->n_infl = n_infl;
        MSB_TRY(ensure_tiles(p));
    }
    return MSB_OK;
}

extern "C" msb_status msb_plan_set_infl(msb_plan p, const double *infl, int n_infl, int per_case) {
    MSB_CHECK(p, MSB_EINVAL, "null plan");
    MSB_CHECK(n_infl == 0 || infl, MSB_EINVAL, "null coefficients");
    return set_infl_many(&p, 1, &infl, n_infl, &per_case);
}
