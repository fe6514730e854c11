// The FFT product f = A u = A_hat u + D^e u + D^f u on a uniform grid, as a chain of
// LDS-staged Stockham passes (Alg. 3 in 2D, Alg. 4 in 3D, re-laid-out for HBM):
//
//   x-forward  : read u rows, zero-pad to Lx, real-to-complex along x (two real rows
//                packed into one complex transform), write the Nx... half spectrum
//                [B][d][Nz][H][Ny] with y contiguous (the column pass reads it whole).
//   2D         : line pass over y: zero-pad Ny -> Ly, FFT, d x d real block product
//                with the generating-array spectra, inverse FFT, keep Ny.
//   3D         : y-forward (to [B][d][H][Ly][Nz], z contiguous), line pass over z
//                with the block product, y-inverse back to [B][d][Nz][H][Ny].
//   x-inverse  : complex-to-real along x, keep Nx, then the sparse corrections
//                D^f (eq. (tea:fr)) and D^e (eq. (tea:sc)), the constraint mask
//                (Sec. 3.4) and a fused epilogue (CG q and p.q, residual, Verlet update).
//
// Zero padding to L >= N + M makes the cyclic product equal the Toeplitz product
// on the grid (the kernel's support is +-M), so only the N first outputs are kept.
#include <cstring>

#include "epilogue.hpp"
#include "fft_device.hpp"
#include "passes.hpp"

namespace msb {

constexpr int kThreads = 256;

__device__ __forceinline__ int comp_of(int a, int b, int d) {
    if (d == 2) return a + b;   // xx=0 xy=1 yy=2
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);   // xx xy xz yy yz zz
}

// Work decomposition.  A block holds a set of signal slots in LDS.  Each slot set
// is processed by a "team": with BLOCK = true the whole block cooperates on all of
// the block's signals (block barriers between Stockham stages, every SIMD busy on a
// few signals: best when there are few signals per CU); with BLOCK = false every
// wavefront owns its own slots and runs all stages with wave-scope ordering only
// (no block barriers: best when there are many signals per CU).
template <bool BLOCK> struct Team {
    int tid, nt;     // thread index within the team, team size
    int w;           // wave index in the block
    __device__ Team() {
        w = threadIdx.x >> 6;
        if (BLOCK) {
            tid = threadIdx.x;
            nt = blockDim.x;
        } else {
            tid = threadIdx.x & 63;
            nt = 64;
        }
    }
    __device__ __forceinline__ void sync() const {
        if (BLOCK) __syncthreads();
        else wave_sync();
    }
    // slot range [s0, s0 + n) of this team, given slots_per_wave in wave mode
    __device__ __forceinline__ void slots(int total, int per_wave, int &s0, int &n) const {
        if (BLOCK) {
            s0 = 0;
            n = total;
        } else {
            s0 = w * per_wave;
            n = max(0, min(per_wave, total - s0));
        }
    }
};

template <typename T, typename T2, int DIR, bool BLOCK, int RMAX>
__device__ __forceinline__ T2 *team_fft(T2 *a, T2 *b, int S, const FftSched &sc, const T2 *tw, const Team<BLOCK> &tm,
                                       bool in_place) {
    // in-place stages (b is not touched and need not exist); only in the kernels with the
    // composite radices, whose register budget already holds 16 values per thread
    if constexpr (RMAX >= 16) {
        if (in_place) {
            fft_inplace<T, T2, DIR, RMAX, BLOCK>(a, S, sc, tw, tm.tid, tm.nt);
            return a;
        }
    }
    if (BLOCK) return fft_lds<T, T2, DIR, RMAX>(a, b, S, sc, tw, tm.tid, tm.nt);
    return fft_wave<T, T2, DIR, RMAX>(a, b, S, sc, tw, tm.tid);
}

// ---------------------------------------------------------------------------- x-forward
// F grid rows per block; complex slot s packs real rows sig = 2s and 2s+1
// (sig = c * nr + r: component c of grid row r0 + r).  Wave mode: each wave owns a.spw consecutive slots.
// tile: this block's tile of the plan's launch (XCD-remapped); ntiles: the plan's
// tile count (the grid of a single-plan launch).
template <typename T, bool BLOCK, int RMAX>
__device__ __forceinline__ void xfwd_body(const PassArgs<T> &a, const EndArgs<T> &e, int tile, int ntiles) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[96];
    const Team<BLOCK> tm;
    const int tpc = (a.rows + a.F - 1) / a.F;
    const int b = tile / tpc;
    const int r0 = (tile - b * tpc) * a.F;
    const int nr = min(a.F, a.rows - r0);
    const int nsig = a.d * nr;
    const int S = (nsig + 1) >> 1;
    const int Lx = a.sx.L;
    const int Smax = (a.d * a.F + 1) >> 1;
    // the previous epilogue's partial sums (cg3): slots per case and array stride
    const int n3 = e.n_cg3 ? e.n_cg3 : tpc;
    const size_t st3 = e.s_cg3 ? e.s_cg3 : (size_t)ntiles;
    T2 *twl = reinterpret_cast<T2 *>(smem);
    T2 *bufA = twl + Lx;
    T2 *bufB = bufA + (size_t)Smax * Lx;
    if (e.done_prev) {
        if (e.done_prev[b]) {   // stopped before this iteration: carry the flag over
            if (r0 == 0 && threadIdx.x == 0) e.done_rw[b] = e.done_prev[b];
            return;
        }
    } else if (e.case_done && e.case_done[b]) {
        return;
    }

    // fused CG step (single reduction per iteration, Chronopoulos-Gear form)
    T alpha = T(0), beta = T(0);
    bool upd = false, conv = false;
    if (e.pro == PRO_CG_P) {
        const int tid0 = threadIdx.x, ntb = blockDim.x;
        if (!e.first) {
            // case sums of r.r, p.q, r.q, q.q: from the per-case reduction when the
            // solver ran one (many tiles per case), else reduced here from the tiles
            double sums[4];
            if (e.case4) {
#pragma unroll
                for (int k = 0; k < 4; ++k) sums[k] = e.case4[(size_t)b * 4 + k];
            } else {
                const double *const parts[4] = {e.rr_prev + (size_t)b * tpc, e.cg3 + (size_t)b * n3,
                                                e.cg3 + st3 + (size_t)b * n3, e.cg3 + 2 * st3 + (size_t)b * n3};
                const int cnt[4] = {tpc, n3, n3, n3};
                block_sum_partials_k<4>(parts, cnt, sums, red, tid0, ntb);
            }
            const double rr = sums[0], pq = sums[1], rq = sums[2], qq = sums[3];
            const double al = rr / pq;
            if (!(pq > 0.0) || !(al == al) || al > 1e300) {   // K not positive definite on p
                if (r0 == 0 && tid0 == 0) e.done_rw[b] = 2;
                return;
            }
            const double rrn = rr - 2.0 * al * rq + al * al * qq;
            if (!(rrn == rrn)) {
                if (r0 == 0 && tid0 == 0) e.done_rw[b] = 3;
                return;
            }
            alpha = T(al);
            beta = T(rr > 0.0 ? rrn / rr : 0.0);
            upd = true;
            conv = e.update_only || (e.thresh && !(rrn > e.thresh[b]));
        } else if (e.beta_num) {
            const double num = block_sum_partials(e.beta_num + (size_t)b * e.n_num, e.n_num, red, tid0, ntb);
            const double den = block_sum_partials(e.beta_den + (size_t)b * e.n_den, e.n_den, red, tid0, ntb);
            beta = T(den > 0.0 ? num / den : 0.0);
        }
    } else if (e.pro == PRO_PCG_R && !e.first) {
        // preconditioned CG: alpha = r.z / p.q; the new r.r = r.r - 2 alpha r.q + alpha^2 q.q
        const int tid0 = threadIdx.x, ntb = blockDim.x;
        double sums[5];
        if (e.case4) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sums[k] = e.case4[(size_t)b * 5 + k];
        } else {
            const double *const parts[5] = {e.rr_prev + (size_t)b * tpc, e.rz_k + (size_t)b * tpc,
                                            e.cg3 + (size_t)b * n3, e.cg3 + st3 + (size_t)b * n3,
                                            e.cg3 + 2 * st3 + (size_t)b * n3};
            const int cnt[5] = {tpc, tpc, n3, n3, n3};
            block_sum_partials_k<5>(parts, cnt, sums, red, tid0, ntb);
        }
        const double rr = sums[0], rz = sums[1], pq = sums[2], rq = sums[3], qq = sums[4];
        const double al = rz / pq;
        if (!(pq > 0.0) || !(rz >= 0.0) || !(al == al) || al > 1e300) {   // K or the preconditioner not SPD
            if (r0 == 0 && tid0 == 0) e.done_rw[b] = 2;
            return;
        }
        const double rrn = rr - 2.0 * al * rq + al * al * qq;
        if (!(rrn == rrn)) {
            if (r0 == 0 && tid0 == 0) e.done_rw[b] = 3;
            return;
        }
        alpha = T(al);
        upd = true;
        conv = e.update_only || (e.thresh && !(rrn > e.thresh[b]));
    } else if (e.pro == PRO_ADR_U && !e.first) {
        // adaptive damping c = 2 sqrt(u.K1.u / u.u) from the previous epilogue's partials;
        // alpha = 2 - c, beta = 1 / (2 + c)
        const int tid0 = threadIdx.x, ntb = blockDim.x;
        double sums[2];
        if (e.case4) {
            sums[0] = e.case4[(size_t)b * 2];
            sums[1] = e.case4[(size_t)b * 2 + 1];
        } else {
            const double *const parts[2] = {e.cg3 + (size_t)b * n3, e.cg3 + st3 + (size_t)b * n3};
            const int cnt[2] = {n3, n3};
            block_sum_partials_k<2>(parts, cnt, sums, red, tid0, ntb);
        }
        const double q = sums[1] > 0.0 ? sums[0] / sums[1] : 0.0;
        const double c = q > 0.0 ? 2.0 * sqrt(q) : 0.0;
        alpha = T(2.0 - c);
        beta = T(1.0 / (2.0 + c));
    } else if (e.pro == PRO_PCG_P && !e.first) {
        // beta = (r.z) / (r.z of the previous iteration)
        const int tid0 = threadIdx.x, ntb = blockDim.x;
        double sums[2];
        if (e.case4) {
            sums[0] = e.case4[(size_t)b * 2];
            sums[1] = e.case4[(size_t)b * 2 + 1];
        } else {
            const double *const parts[2] = {e.rz_k + (size_t)b * tpc, e.rz_km1 + (size_t)b * tpc};
            const int cnt[2] = {tpc, tpc};
            block_sum_partials_k<2>(parts, cnt, sums, red, tid0, ntb);
        }
        beta = T(sums[1] > 0.0 ? sums[0] / sums[1] : 0.0);
    }
    const bool xf = !e.no_transform;
    if (xf) stage_twiddles(twl, a.twx, Lx, threadIdx.x, blockDim.x);
    // whole-workgroup teams: the barrier before the transform also publishes the
    // twiddles, so their loads overlap the data loads; wave teams need it here
    if (!BLOCK) __syncthreads();
    int s0, ns;
    tm.slots(S, a.spw, s0, ns);
    const int nend = xf ? Lx : a.Nx;   // the prologue alone stops at the grid row

    const T hdt2 = T(0.5 * e.dt * e.dt);
    const T dtt = T(e.dt);
    const size_t cbase = (size_t)b * a.d * a.N;
    const FastDiv by_nr((uint32_t)nr, (uint32_t)(2 * S));   // signal -> component (uniform, no division loop)
    double rr_acc = 0.0;
    for (int s = s0; s < s0 + ns; ++s) {
        size_t rowaddr[2];
        int rowfix[2];
        bool has[2];
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
            const int sig = 2 * s + h2;
            has[h2] = sig < nsig;
            const int c = has[h2] ? (int)by_nr.div((uint32_t)sig) : 0;
            const int r = has[h2] ? sig - c * nr : 0;
            rowaddr[h2] = cbase + (size_t)c * a.N + (size_t)(r0 + r) * a.Nx;
            rowfix[h2] = c * a.N + (r0 + r) * a.Nx;
        }
        T2 *dst = bufA + (size_t)s * Lx;
        for (int n = tm.tid; n < nend; n += tm.nt) {
            T2 z;
            z.x = T(0);
            z.y = T(0);
            if (n < a.Nx) {
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    if (!has[h2]) break;
                    const size_t addr = rowaddr[h2] + n;
                    T v;
                    if (e.pro == PRO_NONE) {
                        v = e.pio[addr];
                    } else if (e.pro == PRO_CG_P) {
                        const T pv = e.pio[addr];
                        T rv = e.cr[addr];
                        if (upd) {
                            e.cx[addr] += alpha * pv;
                            rv -= alpha * e.cq[addr];
                            e.cr[addr] = rv;
                        }
                        rr_acc += (double)rv * (double)rv;
                        v = conv ? T(0) : rv + beta * pv;
                        if (!conv) e.pio[addr] = v;
                    } else if (e.pro == PRO_PCG_R) {
                        T rv = e.cr[addr];
                        if (upd) {
                            e.cx[addr] += alpha * e.pr[addr];
                            rv -= alpha * e.cq[addr];
                            e.cr[addr] = rv;
                        }
                        rr_acc += (double)rv * (double)rv;
                        v = conv ? T(0) : rv;
                    } else if (e.pro == PRO_PCG_P) {
                        v = e.pr[addr] + beta * e.pio[addr];
                        e.pio[addr] = v;
                    } else if (e.pro == PRO_ADR_U) {
                        const bool fx = a.fixed && a.fixed[rowfix[h2] + n];
                        T vn = T(0);
                        if (fx) {
                            v = e.pg ? e.pg[addr] : T(0);
                        } else {
                            const T fd = e.cq[addr] / e.pa[addr - cbase + (size_t)b * e.pa_stride];
                            vn = e.first ? T(0.5) * fd : (alpha * e.cx[addr] + T(2) * fd) * beta;
                            v = e.pio[addr] + vn;
                        }
                        e.cx[addr] = vn;
                        e.pio[addr] = v;
                    } else {
                        const bool fx = a.fixed && a.fixed[rowfix[h2] + n];
                        if (fx) v = e.pg ? e.pg[addr] : T(0);
                        else v = e.pio[addr] + dtt * e.pr[addr] + hdt2 * e.pa[addr];
                        e.pio[addr] = v;
                    }
                    if (h2 == 0) z.x = v;
                    else z.y = v;
                }
            }
            if (xf) dst[n] = z;
        }
    }
    if (e.pro == PRO_CG_P || e.pro == PRO_PCG_R) {
        double v[1] = {rr_acc};
        block_sum<1>(v, red, threadIdx.x, blockDim.x);
        if (threadIdx.x == 0) {
            e.rr_out[tile] = v[0];
            if (r0 == 0) {
                if (upd) e.iters[b] += 1;
                if (conv) e.done_rw[b] = e.update_only ? 5 : 1;
                else if (e.done_prev) e.done_rw[b] = 0;
            }
        }
        if (conv) return;
    }
    if (!xf) return;
    tm.sync();
    if (ns > 0) team_fft<T, T2, -1, BLOCK, RMAX>(bufA + (size_t)s0 * Lx, bufB + (size_t)s0 * Lx, ns, a.sx, twl, tm, a.ip_x);
    if (!BLOCK) __syncthreads();
    const T2 *res = (!a.ip_x && (a.sx.np & 1)) ? bufB : bufA;

    // unpack the two real transforms of each slot; x-spectrum k < H into
    // [b][c][z][kx][y].  The whole block stores: thread t owns real row
    // sig = t % nsig and the frequencies kx = t / nsig + j G (G = blockDim / nsig,
    // nsig <= 48 < blockDim), so consecutive threads write consecutive rows of one
    // kx (the transposed layout's contiguous axis) and the loop has no division.
    {
        const int G = blockDim.x / nsig;
        const int sig = threadIdx.x % nsig, k0 = threadIdx.x / nsig;
        if (k0 < G) {
            const int c = sig / nr, row = r0 + sig - c * nr;
            const int z = row / a.Ny, y = row - z * a.Ny;
            T2 *dst = a.T1 + (((size_t)b * a.d + c) * a.Nz + z) * a.H * a.Ny + y;
            const T2 *zs = res + (size_t)(sig >> 1) * Lx;
            const bool odd = (sig & 1) != 0;
            for (int kx = k0; kx < a.H; kx += G) {
                const T2 Z = zs[kx];
                const T2 Zm = zs[kx == 0 ? 0 : Lx - kx];
                T2 X;
                if (!odd) {
                    X.x = T(0.5) * (Z.x + Zm.x);
                    X.y = T(0.5) * (Z.y - Zm.y);
                } else {
                    X.x = T(0.5) * (Z.y + Zm.y);
                    X.y = T(0.5) * (Zm.x - Z.x);
                }
                dst[kx * a.Ny] = X;
            }
        }
    }
}

// ---------------------------------------------------------------------------- line product
// Lines of one case: data[((b*d + c)*nlines + line)*Nl + t], t < Nl.  Fl lines per
// block, slot = (line, component); wave mode: one line (d slots) per wave.  Each
// line is zero-padded to L, transformed, multiplied by the real symmetric d x d
// spectrum block spec[(comp*nlines + line)*L + k] and transformed back.
// zpass = false: the 2D y lines of T1 (nlines = H, length Ny); true: the 3D z lines
// of T2 (nlines = H Ly, length Nz).
template <typename T, bool BLOCK, int RMAX>
__device__ __forceinline__ void line_body(const PassArgs<T> &a, const EndArgs<T> &e, bool zpass, int tile) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const Team<BLOCK> tm;
    T2 *data = zpass ? a.T2 : a.T1;
    const int nlines = zpass ? a.H * a.Ly : a.H;
    const int Nl = zpass ? a.Nz : a.Ny;
    const FftSched &sl = zpass ? a.sz : a.sy;
    const T2 *twg = zpass ? a.twz : a.twy;
    // case-minor tile order: the B cases of a line group are consecutive tiles, which the
    // XCD-contiguous block order runs on one XCD, so the group's spectra are read from
    // HBM once per launch and then served from that XCD's L2 to the other cases
    const int b = tile % a.B;
    const int l0 = (tile / a.B) * a.Fl;
    const int nl = min(a.Fl, nlines - l0);
    const int d = a.d;
    const int L = sl.L;
    T2 *tws = reinterpret_cast<T2 *>(smem);
    T2 *bufA = tws + L;
    T2 *bufB = bufA + (size_t)a.Fl * d * L;
    if (e.case_done && e.case_done[b]) return;
    stage_twiddles(tws, twg, L, threadIdx.x, blockDim.x);
    if (!BLOCK) __syncthreads();   // whole-workgroup teams: published by the barrier before the transform
    int s0, ns;
    tm.slots(nl * d, d * a.lpw, s0, ns);
    if (ns <= 0) return;

    for (int s = s0; s < s0 + ns; ++s) {
        const int li = s / d, c = s - li * d;
        const T2 *src = data + (((size_t)b * d + c) * nlines + l0 + li) * Nl;
        T2 *dst = bufA + (size_t)s * L;
        for (int t = tm.tid; t < L; t += tm.nt) {
            T2 v;
            v.x = T(0);
            v.y = T(0);
            if (t < Nl) v = src[t];
            dst[t] = v;
        }
    }
    const T *spec = a.spec + (size_t)b * a.spec_slot;
    const size_t cstride = (size_t)nlines * L;
    const int lines_here = ns / d;
    // a whole-workgroup team on one line with at most kPf frequencies per thread loads
    // its spectra into registers before the forward transform (their latency hides
    // behind it) instead of between the two transforms
    constexpr int kPf = 2;
    const bool pf = BLOCK && lines_here == 1 && L <= kPf * tm.nt;
    T gpf[kPf][6];
    if (pf) {
        const T *g0 = spec + (size_t)(l0 + s0 / d) * L;
#pragma unroll
        for (int j = 0; j < kPf; ++j) {
            const int k = tm.tid + j * tm.nt;
#pragma unroll
            for (int q = 0; q < 6; ++q) gpf[j][q] = (k < L && q < (d == 2 ? 3 : 6)) ? g0[q * cstride + k] : T(0);
        }
    }
    tm.sync();
    T2 *res = team_fft<T, T2, -1, BLOCK, RMAX>(bufA + (size_t)s0 * L, bufB + (size_t)s0 * L, ns, sl, tws, tm, a.ip_l);
    T2 *oth = (res == bufA + (size_t)s0 * L) ? bufB + (size_t)s0 * L : bufA + (size_t)s0 * L;

    if (pf) {
#pragma unroll
        for (int j = 0; j < kPf; ++j) {
            const int k = tm.tid + j * tm.nt;
            if (k >= L) break;
            T2 *u = res + k;
            if (d == 2) {
                const T gxx = gpf[j][0], gxy = gpf[j][1], gyy = gpf[j][2];
                const T2 ux = u[0], uy = u[L];
                T2 fx, fy;
                fx.x = gxx * ux.x + gxy * uy.x;
                fx.y = gxx * ux.y + gxy * uy.y;
                fy.x = gxy * ux.x + gyy * uy.x;
                fy.y = gxy * ux.y + gyy * uy.y;
                u[0] = fx;
                u[L] = fy;
            } else {
                const T *g = gpf[j];
                const T2 ux = u[0], uy = u[L], uz = u[2 * L];
                T2 fx, fy, fz;
                fx.x = g[0] * ux.x + g[1] * uy.x + g[2] * uz.x;
                fx.y = g[0] * ux.y + g[1] * uy.y + g[2] * uz.y;
                fy.x = g[1] * ux.x + g[3] * uy.x + g[4] * uz.x;
                fy.y = g[1] * ux.y + g[3] * uy.y + g[4] * uz.y;
                fz.x = g[2] * ux.x + g[4] * uy.x + g[5] * uz.x;
                fz.y = g[2] * ux.y + g[4] * uy.y + g[5] * uz.y;
                u[0] = fx;
                u[L] = fy;
                u[2 * L] = fz;
            }
        }
    }
    for (int lk = 0; lk < lines_here && !pf; ++lk)
    for (int k = tm.tid; k < L; k += tm.nt) {
        const int line = l0 + s0 / d + lk;
        const T *g0 = spec + (size_t)line * L + k;
        T2 *u = res + (size_t)lk * d * L + k;
        if (d == 2) {
            const T gxx = g0[0], gxy = g0[cstride], gyy = g0[2 * cstride];
            const T2 ux = u[0], uy = u[L];
            T2 fx, fy;
            fx.x = gxx * ux.x + gxy * uy.x;
            fx.y = gxx * ux.y + gxy * uy.y;
            fy.x = gxy * ux.x + gyy * uy.x;
            fy.y = gxy * ux.y + gyy * uy.y;
            u[0] = fx;
            u[L] = fy;
        } else {
            T g[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) g[q] = g0[q * cstride];
            const T2 ux = u[0], uy = u[L], uz = u[2 * L];
            T2 fx, fy, fz;
            fx.x = g[0] * ux.x + g[1] * uy.x + g[2] * uz.x;
            fx.y = g[0] * ux.y + g[1] * uy.y + g[2] * uz.y;
            fy.x = g[1] * ux.x + g[3] * uy.x + g[4] * uz.x;
            fy.y = g[1] * ux.y + g[3] * uy.y + g[4] * uz.y;
            fz.x = g[2] * ux.x + g[4] * uy.x + g[5] * uz.x;
            fz.y = g[2] * ux.y + g[4] * uy.y + g[5] * uz.y;
            u[0] = fx;
            u[L] = fy;
            u[2 * L] = fz;
        }
    }
    tm.sync();
    T2 *out = team_fft<T, T2, 1, BLOCK, RMAX>(res, oth, ns, sl, tws, tm, a.ip_l);
    for (int s = 0; s < ns; ++s) {
        const int sg = s0 + s;
        const int li = sg / d, c = sg - li * d;
        T2 *dst = data + (((size_t)b * d + c) * nlines + l0 + li) * Nl;
        const T2 *o = out + (size_t)s * L;
        for (int t = tm.tid; t < Nl; t += tm.nt) dst[t] = o[t];
    }
}

// ---------------------------------------------------------------------------- 3D y passes
// y-forward: T1[b][c][z][kx][y<Ny] -> T2[b][c][kx][ky<Ly][z].  Block = Fl consecutive
// z of one (b, kx); slot = (z, component); wave mode: one z-line (d slots) per wave.
template <typename T, bool BLOCK, int RMAX>
__device__ __forceinline__ void yfwd_body(const PassArgs<T> &a, const EndArgs<T> &e, int tile) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const Team<BLOCK> tm;
    const int d = a.d, Ly = a.sy.L;
    const int nzc = (a.Nz + a.Fl - 1) / a.Fl;
    const int tpc = a.H * nzc;
    const int b = tile / tpc;
    const int rem = tile - b * tpc;
    const int kx = rem / nzc;
    const int z0 = (rem - kx * nzc) * a.Fl;
    const int nz = min(a.Fl, a.Nz - z0);
    T2 *twl = reinterpret_cast<T2 *>(smem);
    T2 *bufA = twl + Ly;
    T2 *bufB = bufA + (size_t)a.Fl * d * Ly;
    if (e.case_done && e.case_done[b]) return;
    stage_twiddles(twl, a.twy, Ly, threadIdx.x, blockDim.x);
    if (!BLOCK) __syncthreads();   // whole-workgroup teams: published by the barrier before the transform
    int s0, ns;
    tm.slots(nz * d, d * a.lpw, s0, ns);
    for (int s = s0; s < s0 + ns; ++s) {
        const int zl = s / d, c = s - zl * d;
        const T2 *src = a.T1 + ((((size_t)b * d + c) * a.Nz + z0 + zl) * a.H + kx) * a.Ny;
        T2 *dst = bufA + (size_t)s * Ly;
        for (int t = tm.tid; t < Ly; t += tm.nt) {
            T2 v;
            v.x = T(0);
            v.y = T(0);
            if (t < a.Ny) v = src[t];
            dst[t] = v;
        }
    }
    tm.sync();
    if (ns > 0) team_fft<T, T2, -1, BLOCK, RMAX>(bufA + (size_t)s0 * Ly, bufB + (size_t)s0 * Ly, ns, a.sy, twl, tm, a.ip_l);
    if (!BLOCK) __syncthreads();
    const T2 *res = (!a.ip_l && (a.sy.np & 1)) ? bufB : bufA;
    // the whole block stores: thread t owns z = z0 + t % nz and ky = t / nz + j G
    // (G = blockDim / nz, nz <= 16 < blockDim), consecutive threads on consecutive z
    // (T2's contiguous axis)
    {
        const int G = blockDim.x / nz;
        const int zl = threadIdx.x % nz, k0 = threadIdx.x / nz;
        if (k0 < G) {
            for (int c = 0; c < d; ++c) {
                T2 *dst = a.T2 + (((size_t)b * d + c) * a.H + kx) * Ly * a.Nz + z0 + zl;
                const T2 *src = res + (size_t)(zl * d + c) * Ly;
                for (int ky = k0; ky < Ly; ky += G) dst[ky * a.Nz] = src[ky];
            }
        }
    }
}

// y-inverse: T2[b][c][kx][ky][z] -> T1[b][c][z][kx][y<Ny]
template <typename T, bool BLOCK, int RMAX>
__device__ __forceinline__ void yinv_body(const PassArgs<T> &a, const EndArgs<T> &e, int tile) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const Team<BLOCK> tm;
    const int d = a.d, Ly = a.sy.L;
    const int nzc = (a.Nz + a.Fl - 1) / a.Fl;
    const int tpc = a.H * nzc;
    const int b = tile / tpc;
    const int rem = tile - b * tpc;
    const int kx = rem / nzc;
    const int z0 = (rem - kx * nzc) * a.Fl;
    const int nz = min(a.Fl, a.Nz - z0);
    T2 *twl = reinterpret_cast<T2 *>(smem);
    T2 *bufA = twl + Ly;
    T2 *bufB = bufA + (size_t)a.Fl * d * Ly;
    if (e.case_done && e.case_done[b]) return;
    stage_twiddles(twl, a.twy, Ly, threadIdx.x, blockDim.x);   // published by the barrier after the gather
    int s0, ns;
    tm.slots(nz * d, d * a.lpw, s0, ns);
    {
        // the whole block loads: thread t owns z = z0 + t % nz and ky = t / nz + j G,
        // consecutive threads on consecutive z
        const int G = blockDim.x / nz;
        const int zl = threadIdx.x % nz, k0 = threadIdx.x / nz;
        if (k0 < G) {
            for (int c = 0; c < d; ++c) {
                const T2 *src = a.T2 + (((size_t)b * d + c) * a.H + kx) * Ly * a.Nz + z0 + zl;
                T2 *dst = bufA + (size_t)(zl * d + c) * Ly;
                for (int ky = k0; ky < Ly; ky += G) dst[ky] = src[ky * a.Nz];
            }
        }
    }
    __syncthreads();
    if (ns <= 0) return;
    T2 *res = team_fft<T, T2, 1, BLOCK, RMAX>(bufA + (size_t)s0 * Ly, bufB + (size_t)s0 * Ly, ns, a.sy, twl, tm, a.ip_l);
    for (int s = 0; s < ns; ++s) {
        const int sg = s0 + s;
        const int zl = sg / d, c = sg - zl * d;
        T2 *dst = a.T1 + ((((size_t)b * d + c) * a.Nz + z0 + zl) * a.H + kx) * a.Ny;
        const T2 *o = res + (size_t)s * Ly;
        for (int t = tm.tid; t < a.Ny; t += tm.nt) dst[t] = o[t];
    }
}

// ---------------------------------------------------------------------------- x-inverse
// Slots as in the x-forward pass.  Each slot's full x-spectrum is rebuilt from the
// half spectra of its two real rows, transformed back, then the broken-bond
// correction of those rows, the incomplete-horizon diagonal, the constraint mask and
// the fused epilogue are applied.
template <typename T, bool BLOCK, int RMAX>
__device__ __forceinline__ void xinv_body(const PassArgs<T> &a, const EndArgs<T> &e, int tile, int ntiles) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[96];
    const Team<BLOCK> tm;
    const int tpc = (a.rows + a.F - 1) / a.F;
    const int b = tile / tpc;
    const int r0 = (tile - b * tpc) * a.F;
    const int nr = min(a.F, a.rows - r0);
    const int d = a.d;
    const int nsig = d * nr;
    const int S = (nsig + 1) >> 1;
    const int Lx = a.sx.L;
    const int Smax = (d * a.F + 1) >> 1;
    T2 *twl = reinterpret_cast<T2 *>(smem);
    T2 *bufA = twl + Lx;
    T2 *bufB = bufA + (size_t)Smax * Lx;
    if (e.case_done && e.case_done[b]) return;
    // uniform splits signal -> (component, row) and row -> (z, y) by multiply-high: the
    // per-slot loops below would otherwise run a scalar division sequence each time
    const FastDiv by_nr((uint32_t)nr, (uint32_t)(2 * S));
    const FastDiv by_ny((uint32_t)a.Ny, (uint32_t)a.rows);
    stage_twiddles(twl, a.twx, Lx, threadIdx.x, blockDim.x);   // published by the barrier after the gather
    // the constraint class of each signal's x-row (published by the same barrier), so that the
    // epilogue neither waits for it nor reads the mask of rows with none or all constrained
    __shared__ uint8_t rfl[48];   // d F signals: F <= 16 rows per workgroup, d <= 3
    for (int t = threadIdx.x; t < nsig; t += blockDim.x) {
        const int c = (int)by_nr.div((uint32_t)t), row = r0 + t - c * nr;
        rfl[t] = a.fixed ? a.row_fix[(size_t)c * a.rows + row] : 0;
    }
    int s0, ns;
    tm.slots(S, a.spw_i, s0, ns);

    // full spectrum Z = Xa + i Xb of every slot with the Hermitian halves mirrored.
    // The whole block loads: thread t owns slot sl = t % S and the frequencies
    // kx = t / S + j G (G = blockDim / S, S <= 24 < blockDim); consecutive threads
    // read consecutive rows of one kx, no division in the loop.
    {
        const int G = blockDim.x / S;
        const int sl = threadIdx.x % S, k0 = threadIdx.x / S;
        if (k0 < G) {
            const T2 *src[2] = {nullptr, nullptr};
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const int sig = 2 * sl + h2;
                if (sig < nsig) {
                    const int c = sig / nr, row = r0 + sig - c * nr;
                    const int z = row / a.Ny, y = row - z * a.Ny;
                    src[h2] = a.T1 + (((size_t)b * d + c) * a.Nz + z) * a.H * a.Ny + y;
                }
            }
            T2 *zs = bufA + (size_t)sl * Lx;
            for (int kx = k0; kx < a.H; kx += G) {
                T2 X0, X1;
                X0.x = X0.y = X1.x = X1.y = T(0);
                if (src[0]) X0 = src[0][kx * a.Ny];
                if (src[1]) X1 = src[1][kx * a.Ny];
                T2 Z;
                Z.x = X0.x - X1.y;
                Z.y = X0.y + X1.x;
                zs[kx] = Z;
                const int m = Lx - kx;
                if (kx >= 1 && m >= a.H) {
                    T2 Zm;
                    Zm.x = X0.x + X1.y;
                    Zm.y = -X0.y + X1.x;
                    zs[m] = Zm;
                }
            }
        }
    }
    __syncthreads();
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    if (ns > 0) {
        const int nsg = min(2 * ns, nsig - 2 * s0);   // real rows of this team
        const size_t cbase = (size_t)b * d * a.N;
        const T *uin = e.uin;
        T2 *R = team_fft<T, T2, 1, BLOCK, RMAX>(bufA + (size_t)s0 * Lx, bufB + (size_t)s0 * Lx, ns, a.sx, twl, tm, a.ip_x);
        T *Rr = reinterpret_cast<T *>(R);   // real row sl of this team at Rr[2 ((sl>>1) Lx + n) + (sl&1)]

        const int M = a.M, M1 = a.M + 1;
        const bool narrow = a.Nx <= 2 * M;   // every column is within M of an x face
        // broken bonds (eq. (tea:fr)): f_p += sum_{q in v_p} W(q - p) (u_p - u_q); with
        // the surface correction a bond of a row of Omega_e carries v_pq W, so v_pq W
        // is removed
        if (a.br_row_ptr && a.corr) {
            const T *wt = a.w + (size_t)b * a.w_slot;
            for (int sl = 0; sl < nsg; ++sl) {
                const int sig = 2 * s0 + sl;
                const int c = (int)by_nr.div((uint32_t)sig), row = r0 + sig - c * nr;
                const int z = (int)by_ny.div((uint32_t)row), y = row - z * a.Ny;
                const bool row_e = y < M || y >= a.Ny - M || (d == 3 && (z < M || z >= a.Nz - M));
                const int e0 = a.br_row_ptr[row], e1 = a.br_row_ptr[row + 1];
                for (int ei = e0 + tm.tid; ei < e1; ei += tm.nt) {
                    const int node = a.br_node_i[ei];
                    const int n = node - row * a.Nx;
                    const bool on_e = a.nu && (row_e || n < M || n >= a.Nx - M);
                    const double nup = on_e ? (double)a.nu[node] : 0.0;
                    // the node's bonds four at a time (their index, u and weight loads in
                    // flight together: a node has about ten broken bonds at a crack), four
                    // partial sums added in a fixed order
                    constexpr int kU = 4;
                    double up[3] = {0.0, 0.0, 0.0};
                    for (int cb = 0; cb < d; ++cb) up[cb] = (double)uin[cbase + (size_t)cb * a.N + node];
                    double part[kU] = {0.0, 0.0, 0.0, 0.0};
                    const int tb1 = a.br_bond_ptr[ei + 1];
                    for (int t0 = a.br_bond_ptr[ei]; t0 < tb1; t0 += kU) {
                        int q[kU], o[kU];
#pragma unroll
                        for (int k = 0; k < kU; ++k) {
                            const bool ok = t0 + k < tb1;
                            q[k] = ok ? a.br_q[t0 + k] : node;   // a missing bond reads node p: du = 0
                            o[k] = ok ? a.br_off[t0 + k] : 0;
                        }
#pragma unroll
                        for (int k = 0; k < kU; ++k) {
                            double wb = 0.0;
                            for (int cb = 0; cb < d; ++cb) {
                                const double du = up[cb] - (double)uin[cbase + (size_t)cb * a.N + q[k]];
                                wb += (double)wt[(size_t)comp_of(c, cb, d) * a.n_off + o[k]] * du;
                            }
                            part[k] += on_e ? 0.5 * (nup + (double)a.nu[q[k]]) * wb : wb;
                        }
                    }
                    const double accb = (part[0] + part[1]) + (part[2] + part[3]);
                    Rr[2 * ((size_t)(sl >> 1) * Lx + n) + (sl & 1)] += T(accb);
                }
            }
            tm.sync();
        }

        // incomplete horizon (eq. (tea:sc)): f += D^e u with D^e from the table indexed
        // by the clamped distances to the faces.  Applied to the rows in LDS before the
        // epilogue, as its own pass: an interior row needs it only on its first and
        // last M columns, so those are gathered across all rows of the team in one
        // flat loop (one memory round trip for the team instead of one per row).
        const T *de = a.de + (size_t)b * a.de_slot;
        // table index = (lx (M+1) + hx) (M+1)^(2d-2) + [y and z part, fixed per row]
        const int M1p = d == 2 ? M1 * M1 : M1 * M1 * M1 * M1;
        auto row_of = [&](int sl, int &c, int &row, int &rpart) -> bool {
            const int sig = 2 * s0 + sl;
            c = (int)by_nr.div((uint32_t)sig);
            row = r0 + sig - c * nr;
            const int z = (int)by_ny.div((uint32_t)row), y = row - z * a.Ny;
            const int ly = min(y, M), hy = min(a.Ny - 1 - y, M);
            const int lz = d == 3 ? min(z, M) : 0, hz = d == 3 ? min(a.Nz - 1 - z, M) : 0;
            rpart = ly * M1 + hy;
            if (d == 3) rpart = (rpart * M1 + lz) * M1 + hz;
            return (ly == M) & (hy == M) & (d == 2 || ((lz == M) & (hz == M)));   // interior row
        };
        auto apply_de = [&](int sl, int c, int row, int rpart, int n) {
            const int lx = min(n, M), hx = min(a.Nx - 1 - n, M);
            const int dx = (lx * M1 + hx) * M1p + rpart;
            const T *urow = uin + cbase + (size_t)row * a.Nx + n;   // component cb at urow[cb N]
            T *fr = Rr + 2 * ((size_t)(sl >> 1) * Lx + n) + (sl & 1);
            T f = *fr;
            for (int cb = 0; cb < d; ++cb) f += de[(size_t)comp_of(c, cb, d) * a.de_stride + dx] * urow[(size_t)cb * a.N];
            *fr = f;
        };
        // surface correction (Remark 3, eq. (scr)): on the nodes of Omega_e (within M of
        // a face) every bond is scaled by v_pq = (nu_p + nu_q) / 2, i.e. f_p +=
        // sum_o (v_pq - 1) W(o) (u_{p+o} - u_p) over the neighbours inside the grid
        // (broken ones included: the D^f term above removed v_pq W for those)
        if (a.nu && a.corr) {
            const T *wt = a.w + (size_t)b * a.w_slot;
            for (int sl = 0; sl < nsg; ++sl) {
                int c, row, rpart;
                const bool edge_cols = row_of(sl, c, row, rpart) && !narrow;   // interior row
                const int z = (int)by_ny.div((uint32_t)row), y = row - z * a.Ny;
                const int ncol = edge_cols ? 2 * M : a.Nx;
                for (int jj = tm.tid; jj < ncol; jj += tm.nt) {
                    const int n = edge_cols ? (jj < M ? jj : a.Nx - 2 * M + jj) : jj;
                    const int node = row * a.Nx + n;
                    const double nup = (double)a.nu[node];
                    double acc = 0.0;
                    for (int o = 0; o < a.n_off; ++o) {
                        const int ox = a.offs[3 * o], oy = a.offs[3 * o + 1], oz = a.offs[3 * o + 2];
                        const int xx = n + ox, yy = y + oy, zz = z + oz;
                        if (xx < 0 || xx >= a.Nx || yy < 0 || yy >= a.Ny || zz < 0 || zz >= a.Nz) continue;
                        const int q = node + (oz * a.Ny + oy) * a.Nx + ox;
                        double wb = 0.0;
                        for (int cb = 0; cb < d; ++cb) {
                            const double du = (double)uin[cbase + (size_t)cb * a.N + q] -
                                              (double)uin[cbase + (size_t)cb * a.N + node];
                            wb += (double)wt[(size_t)comp_of(c, cb, d) * a.n_off + o] * du;
                        }
                        acc += (0.5 * (nup + (double)a.nu[q]) - 1.0) * wb;
                    }
                    Rr[2 * ((size_t)(sl >> 1) * Lx + n) + (sl & 1)] += T(acc);
                }
            }
            tm.sync();
        }
        // (whole-workgroup teams apply D^e inline in the epilogue instead: there only
        // the waves holding boundary columns wait for the table, with no extra barrier)
        if (!BLOCK && !narrow && a.corr) {
            // interior rows: columns [0, M) and [Nx - M, Nx), flattened over the rows
            const int per = 2 * M;
            for (int jj = tm.tid; jj < nsg * per; jj += tm.nt) {
                const int sl = jj / per, j = jj - sl * per;
                int c, row, rpart;
                if (!row_of(sl, c, row, rpart)) continue;
                apply_de(sl, c, row, rpart, j < M ? j : a.Nx - per + j);
            }
        }
        // rows within M of a y or z face (or every row of a narrow grid): all columns
        for (int sl = 0; sl < nsg && !BLOCK && a.corr; ++sl) {
            int c, row, rpart;
            if (row_of(sl, c, row, rpart) && !narrow) continue;
#pragma unroll 4
            for (int n = tm.tid; n < a.Nx; n += tm.nt) apply_de(sl, c, row, rpart, n);
        }
        if (!BLOCK) tm.sync();

        const T dth = T(0.5 * e.dt);
        const T rinv = T(1.0 / e.rho);
        const T sign = T(e.sign);
        for (int sl = 0; sl < nsg; ++sl) {
            int c, row, rpart;
            const bool rint = row_of(sl, c, row, rpart);
            const size_t rbase = cbase + (size_t)c * a.N + (size_t)row * a.Nx;
            // the mask is read only on x-rows with some (not all) DOFs constrained
            const int rf = rfl[2 * s0 + sl];
            const uint8_t *fxrow = rf == 2 ? a.fixed + (size_t)c * a.N + (size_t)row * a.Nx : nullptr;
            const T *Rrow = Rr + 2 * (size_t)(sl >> 1) * Lx + (sl & 1);
            const T *dec[3];
            for (int cb = 0; cb < 3; ++cb) dec[cb] = de + (size_t)comp_of(c, cb < d ? cb : 0, d) * a.de_stride + rpart;
            const T *urow = uin + cbase + (size_t)row * a.Nx;   // component cb at urow[cb N + n]
            for (int n = tm.tid; n < a.Nx; n += tm.nt) {
                const size_t addr = rbase + n;
                T f = Rrow[2 * n];
                if (BLOCK && a.corr) {
                    const int lx = min(n, M), hx = min(a.Nx - 1 - n, M);
                    if (!(rint & (lx == M) & (hx == M))) {
                        const int dx = (lx * M1 + hx) * M1p;
                        for (int cb = 0; cb < d; ++cb) f += dec[cb][dx] * urow[cb * a.N + n];
                    }
                }
                const bool fx = rf == 1 || (fxrow && fxrow[n]);
                epilogue_at<T>(e, uin, addr, addr - cbase + (size_t)b * e.pa_stride, f, fx, sign, rinv, dth, acc0, acc1,
                               acc2);
            }
        }
    }
    if (e.part) {
        double v[3] = {acc0, acc1, acc2};
        block_sum<3>(v, red, threadIdx.x, blockDim.x);
        if (threadIdx.x == 0) {
            const size_t stride = (size_t)ntiles;
            e.part[tile] = v[0];
            e.part[stride + tile] = v[1];
            e.part[2 * stride + tile] = v[2];
        }
    }
}

// ---------------------------------------------------------------------------- kernels
// Single-plan launches: the grid is the plan's tiles, remapped so that the blocks of
// one XCD take a contiguous tile range.  Group launches: one grid over the tiles of
// several plans; each block finds its plan in start[] (group_member) after the same
// remap and takes that plan's arguments from device arrays.

#define MSB_PLAN_KERNEL(NAME, BODY, ...)                                                              \
    template <typename T, bool BLOCK, int RMAX>                                                      \
    __global__ __launch_bounds__(kMaxBlock) void NAME(PassArgs<T> a, EndArgs<T> e) {                      \
        const int tile = xcd_tile(blockIdx.x, gridDim.x), ntiles = gridDim.x;                        \
        (void)ntiles;                                                                                \
        BODY<T, BLOCK, RMAX>(a, e, __VA_ARGS__);                                                     \
    }                                                                                                \
    template <typename T, bool BLOCK, int RMAX>                                                      \
    __global__ __launch_bounds__(kMaxBlock) void NAME##_group(const PassArgs<T> *__restrict__ A,          \
                                                         const EndArgs<T> *__restrict__ E,           \
                                                         const int *__restrict__ start, int n) {    \
        const int g = xcd_tile(blockIdx.x, gridDim.x);                                               \
        const int m = group_member(start, n, g);                                                     \
        const int tile = g - start[m], ntiles = start[m + 1] - start[m];                             \
        (void)ntiles;                                                                                \
        BODY<T, BLOCK, RMAX>(A[m], E[m], __VA_ARGS__);                                               \
    }

MSB_PLAN_KERNEL(k_xfwd, xfwd_body, tile, ntiles)
MSB_PLAN_KERNEL(k_line_y, line_body, false, tile)
MSB_PLAN_KERNEL(k_line_z, line_body, true, tile)
MSB_PLAN_KERNEL(k_yfwd, yfwd_body, tile)
MSB_PLAN_KERNEL(k_yinv, yinv_body, tile)
MSB_PLAN_KERNEL(k_xinv, xinv_body, tile, ntiles)

// ---------------------------------------------------------------------------- host side
int x_tiles_per_case(const msb_plan_s *p, int F) { return (int)((rows_total(p) + F - 1) / F); }

// LDS bytes: the shared twiddle table plus two buffers (ping-pong) of slots.
// twiddles plus two signal buffers (one with in-place stages)
static size_t lds_x_bytes(int d, int F, int64_t Lx, size_t cbytes, bool in_place = false) {
    return ((size_t)(in_place ? 1 : 2) * ((d * F + 1) / 2) + 1) * Lx * cbytes;
}
static size_t lds_line_bytes(int d, int Fl, int64_t L, size_t cbytes, bool in_place = false) {
    return ((size_t)(in_place ? 1 : 2) * Fl * d + 1) * L * cbytes;
}
static int waves_x(int d, int F) { return (d * F + 1) / 2; }
// tiled product: twiddles plus two tl x (tl | 1) frames
static size_t lds_tile_bytes(int tl, size_t cbytes) { return ((size_t)tl + 2 * (size_t)tl * (tl | 1)) * cbytes; }
// frame lengths of the tiled product and the smallest inner block per axis
constexpr int kTileMin = 8, kTileMax64 = 64, kTileMax32 = 96, kTileInnerMin = 4;

// Dynamic LDS a workgroup may use (gfx950: 160 KiB per workgroup, less the
// kernels' static reduction scratch), and the budget the default configuration
// keeps to so that two workgroups fit on a CU.
constexpr size_t kLdsMax = 160 * 1024 - 1024;
constexpr size_t kLdsDefault = 80 * 1024;

static int64_t x_units(const msb_plan_s *p) { return (int64_t)p->B * ((rows_total(p) * p->dim + 1) / 2); }
static int64_t line_count(const msb_plan_s *p) { return p->dim == 2 ? p->H : p->H * p->n[2]; }
static int64_t line_len(const msb_plan_s *p) { return p->dim == 2 ? p->L[1] : std::max(p->L[1], p->L[2]); }

// Default configuration.  Team choice: wave-owned signals once there are enough
// independent signals to give every SIMD of the chip (256 CUs x 4) several of them,
// whole-workgroup teams otherwise.  x passes: the largest power of two <= 8 rows
// per workgroup within the LDS budget (4 for FP32 wave teams, which own several
// slots per wave), and >= 1024 workgroups for block teams (latency-bound small
// grids run fastest with few rows per workgroup).  Line passes: up to 8 lines per
// workgroup, >= 256 workgroups for block teams.
msb_launch_config default_config(const msb_plan_s *p, bool fp32) {
    msb_launch_config c;
    const size_t cb = fp32 ? sizeof(float2) : sizeof(double2);
    const int d = p->dim;
    const int64_t rows = rows_total(p);
    c.team_x = x_units(p) >= 4096 ? 1 : 0;
    int F = c.team_x && fp32 ? 4 : 8;
    const int wslots = c.team_x && fp32 ? 2 : 1;   // the smaller of the two slot counts below
    while (F > 1 && (lds_x_bytes(d, F, p->L[0], cb) > kLdsDefault || waves_x(d, F) > (kMaxBlock / 64) * wslots ||
                     (!c.team_x && (int64_t)p->B * ((rows + F - 1) / F) < 1024)))
        F /= 2;
    c.rows_per_wg = F;
    c.slots_fwd = c.team_x && fp32 ? 4 : 1;
    c.slots_inv = c.team_x && fp32 ? 2 : 1;
    c.threads_x = 256;
    const int64_t nl = line_count(p), Ll = line_len(p);
    c.team_line = (int64_t)p->B * nl >= 4096 ? 1 : 0;
    int Fl = 8;
    while (Fl > 1 && (lds_line_bytes(d, Fl, Ll, cb) > kLdsDefault ||
                      (!c.team_line && (int64_t)p->B * ((nl + Fl - 1) / Fl) < 256)))
        Fl /= 2;
    c.lines_per_wg = Fl;
    c.lines_per_wave = 1;
    // 2D block teams: about one thread per 4 points of the workgroup's signals
    c.threads_line = (d == 2 && (int64_t)Fl * d * Ll >= 2048) ? 512 : 256;
    c.max_radix = fp32 ? 16 : 8;
    c.lds_inplace = 0;
    c.tile = 0;
    c.threads_tile = 256;
    c.tile_regs = 0;
    c.tile_run = 1;
    return c;
}

// In-place stages keep all of a thread's butterflies of a stage in registers: for S
// signals on nt threads, at most inplace_batch(R, RMAX) per thread in every stage
// (RMAX of the kernel the plan's schedules select: 16 with composite radices, else 8;
// a group may run the plan in a 16 kernel, whose bound is not smaller).
static bool inplace_fits(const FftSched &s, int64_t S, int64_t nt, int rmax) {
    for (int i = 0; i < s.np; ++i)
        if ((S * s.ps[i].nb + nt - 1) / nt > inplace_batch(s.ps[i].R, rmax)) return false;
    return true;
}

// Exactness of the Stockham index split: fdiv(t, nb) with t < S * nb is exact while
// S * nb^2 < 2^32 (S = signals a team transforms together).
static bool split_exact(int64_t S, int64_t L) {
    const int64_t nb = L / 2;   // largest butterfly count of any stage (radix >= 2)
    return S * nb * nb < (int64_t(1) << 32);
}

msb_status check_config(const msb_plan_s *p, bool fp32, const msb_launch_config &c) {
    const size_t cb = fp32 ? sizeof(float2) : sizeof(double2);
    const int d = p->dim;
    MSB_CHECK(c.rows_per_wg >= 1 && c.rows_per_wg <= 16, MSB_EINVAL, "rows_per_wg %d not in [1, 16]", c.rows_per_wg);
    MSB_CHECK(c.lines_per_wg >= 1 && c.lines_per_wg <= 16, MSB_EINVAL, "lines_per_wg %d not in [1, 16]", c.lines_per_wg);
    MSB_CHECK((c.team_x == 0 || c.team_x == 1) && (c.team_line == 0 || c.team_line == 1), MSB_EINVAL,
              "team_x / team_line must be 0 or 1");
    MSB_CHECK(c.slots_fwd >= 1 && c.slots_fwd <= 8 && c.slots_inv >= 1 && c.slots_inv <= 8, MSB_EINVAL,
              "slots_fwd / slots_inv not in [1, 8]");
    MSB_CHECK(c.lines_per_wave >= 1 && c.lines_per_wave <= 8, MSB_EINVAL, "lines_per_wave not in [1, 8]");
    for (int t : {c.threads_x, c.threads_line})
        MSB_CHECK(t >= 64 && t <= kMaxBlock && t % 64 == 0, MSB_EINVAL, "thread count %d: need a multiple of 64 in [64, %d]",
                  t, kMaxBlock);
    MSB_CHECK(c.max_radix == 4 || c.max_radix == 8 || c.max_radix == 16, MSB_EINVAL, "max_radix must be 4, 8 or 16");
    MSB_CHECK(c.lds_inplace >= 0 && c.lds_inplace <= 3, MSB_EINVAL, "lds_inplace must be in [0, 3]");
    const bool ipx = (c.lds_inplace & 1) != 0, ipl = (c.lds_inplace & 2) != 0;
    if (ipx || ipl) {
        const FftSched sx = make_sched(p->ax[0], fp32, c.max_radix), sy = make_sched(p->ax[1], fp32, c.max_radix),
                       sz = make_sched(p->ax[2], fp32, c.max_radix);
        const int rk = plan_needs_composite(p, fp32, c.max_radix) ? 16 : 8;
        MSB_CHECK(rk == 16, MSB_EINVAL, "lds_inplace needs a schedule with a composite radix (max_radix 16 and "
                  "a length that uses one)");
        const int64_t Sx = c.team_x ? std::max(c.slots_fwd, c.slots_inv) : waves_x(d, c.rows_per_wg);
        const int64_t ntx = c.team_x ? 64 : c.threads_x;
        const int64_t Sl = (int64_t)d * (c.team_line ? c.lines_per_wave : c.lines_per_wg);
        const int64_t ntl = c.team_line ? 64 : c.threads_line;
        MSB_CHECK(!ipx || inplace_fits(sx, Sx, ntx, rk), MSB_EINVAL,
                  "lds_inplace: an x-pass thread would own more butterflies of a stage than it holds in registers");
        MSB_CHECK(!ipl || (d == 2 ? inplace_fits(sy, Sl, ntl, rk) : inplace_fits(sz, Sl, ntl, rk) && inplace_fits(sy, Sl, ntl, rk)),
                  MSB_EINVAL, "lds_inplace: a line-pass thread would own more butterflies of a stage than it holds in registers");
    }
    const size_t lx = lds_x_bytes(d, c.rows_per_wg, p->L[0], cb, ipx);
    MSB_CHECK(lx <= kLdsMax, MSB_EINVAL, "x passes need %zu bytes of LDS per workgroup (max %zu)", lx, kLdsMax);
    const size_t ll = lds_line_bytes(d, c.lines_per_wg, line_len(p), cb, ipl);
    MSB_CHECK(ll <= kLdsMax, MSB_EINVAL, "line passes need %zu bytes of LDS per workgroup (max %zu)", ll, kLdsMax);
    if (c.team_x) {
        const int w = waves_x(d, c.rows_per_wg);
        MSB_CHECK(64 * ((w + c.slots_fwd - 1) / c.slots_fwd) <= kMaxBlock &&
                      64 * ((w + c.slots_inv - 1) / c.slots_inv) <= kMaxBlock,
                  MSB_EINVAL, "x passes: %d slots need more than %d waves per workgroup", w, kMaxBlock / 64);
    }
    MSB_CHECK(64 * ((c.lines_per_wg + c.lines_per_wave - 1) / c.lines_per_wave) <= kMaxBlock, MSB_EINVAL,
              "line passes: too many waves per workgroup");
    const int64_t sx = c.team_x ? std::max(c.slots_fwd, c.slots_inv) : waves_x(d, c.rows_per_wg);
    const int64_t sl = c.team_line ? (int64_t)d * c.lines_per_wave : (int64_t)d * c.lines_per_wg;
    MSB_CHECK(split_exact(sx, p->L[0]) && split_exact(sl, line_len(p)), MSB_EINVAL,
              "too many signals per team for the transform length");
    MSB_CHECK(c.threads_tile >= 64 && c.threads_tile <= kMaxBlock && c.threads_tile % 64 == 0, MSB_EINVAL,
              "threads_tile %d: need a multiple of 64 in [64, %d]", c.threads_tile, kMaxBlock);
    if (c.tile != 0) {
        MSB_CHECK(d == 2, MSB_EINVAL, "the tiled product is 2D only (tile must be 0)");
        const int tmax = fp32 ? kTileMax32 : kTileMax64;
        MSB_CHECK(c.tile >= kTileMin && c.tile <= tmax, MSB_EINVAL, "tile %d not in [%d, %d]", c.tile, kTileMin, tmax);
        std::vector<int> r;
        MSB_CHECK(factor_length(c.tile, r, 16), MSB_EINVAL, "tile %d has a prime factor above 5", c.tile);
        MSB_CHECK(c.tile - 2 * p->M >= kTileInnerMin, MSB_EINVAL, "tile %d leaves fewer than %d inner nodes per axis at M = %d",
                  c.tile, kTileInnerMin, p->M);
        const size_t lt = lds_tile_bytes(c.tile, cb);
        MSB_CHECK(lt <= kLdsMax, MSB_EINVAL, "tile %d needs %zu bytes of LDS per workgroup (max %zu)", c.tile, lt, kLdsMax);
    }
    MSB_CHECK(c.tile_regs == 0 || c.tile_regs == 1, MSB_EINVAL, "tile_regs %d: need 0 or 1", c.tile_regs);
    MSB_CHECK(!c.tile_regs || c.tile == 16 || c.tile == 32 || c.tile == 64, MSB_EINVAL,
              "tile_regs = 1 needs tile 16, 32 or 64 (got %d)", c.tile);
    MSB_CHECK(c.tile_run >= 1 && c.tile_run <= 64, MSB_EINVAL, "tile_run %d not in [1, 64]", c.tile_run);
    return MSB_OK;
}

int tile_count(const msb_plan_s *p, int tl) {
    if (tl <= 0) return 0;
    const int64_t T = tl - 2 * p->M;
    return (int)(((p->n[0] + T - 1) / T) * ((p->n[1] + T - 1) / T));
}

int64_t partial_slots(const msb_plan_s *p) {
    int64_t s = rows_total(p);
    if (p->dim == 2) {
        const int64_t T = kTileInnerMin;
        s = std::max<int64_t>(s, ((p->n[0] + T - 1) / T) * ((p->n[1] + T - 1) / T));
    }
    return s;
}

template <typename T> static const T *sel(const double *a, const float *b);
template <> const double *sel<double>(const double *a, const float *) { return a; }
template <> const float *sel<float>(const double *, const float *b) { return b; }

template <typename T> PassArgs<T> pass_args(const msb_plan_s *p, const DeviceOp &op, const msb_launch_config *cfg) {
    PassArgs<T> a;
    memset(&a, 0, sizeof(a));   // padding zero: argument blocks compare bytewise (cached solver graphs)
    const bool f32 = sizeof(T) == 4;
    a.d = p->dim;
    a.B = p->B;
    a.Nx = (int)p->n[0];
    a.Ny = (int)p->n[1];
    a.Nz = (int)p->n[2];
    a.M = p->M;
    a.rows = (int)rows_total(p);
    a.H = (int)p->H;
    a.Ly = (int)p->L[1];
    a.Lz = (int)p->L[2];
    a.N = (int)p->N;
    a.corr = 1;
    const msb_launch_config &c = cfg ? *cfg : p->cfg[f32 ? 1 : 0];
    a.F = c.rows_per_wg;
    a.Fl = c.lines_per_wg;
    a.wave_x = c.team_x;
    a.wave_l = c.team_line;
    a.spw = c.slots_fwd;
    a.spw_i = c.slots_inv;
    a.lpw = c.lines_per_wave;
    a.ip_x = c.lds_inplace & 1;
    a.ip_l = (c.lds_inplace >> 1) & 1;
    a.bthreads = c.threads_x;
    a.bthreads_line = c.threads_line;
    if (cfg) {   // the given configuration's radix cap, not the plan's
        a.sx = make_sched(p->ax[0], f32, c.max_radix);
        a.sy = make_sched(p->ax[1], f32, c.max_radix);
        a.sz = make_sched(p->ax[2], f32, c.max_radix);
    } else {
        a.sx = sched_of(p->ax[0], f32);
        a.sy = sched_of(p->ax[1], f32);
        a.sz = sched_of(p->ax[2], f32);
    }
    a.twx = tw_of<T>(p->ax[0]);
    a.twy = tw_of<T>(p->ax[1]);
    a.twz = tw_of<T>(p->ax[2]);
    a.T1 = reinterpret_cast<cplx_t<T> *>(p->T1);
    a.T2 = reinterpret_cast<cplx_t<T> *>(p->T2);
    a.spec = sel<T>(op.spec64, op.spec32);
    a.de = sel<T>(op.de64, op.de32);
    a.w = sel<T>(op.w64, op.w32);
    const bool multi = op.count > 1;
    a.spec_slot = multi ? (size_t)p->ncomp * spectrum_len(p) : 0;
    a.de_slot = multi ? de_len(p) : 0;
    a.w_slot = multi ? w_len(p) : 0;
    a.de_stride = p->de_stride;
    a.n_off = p->n_off;
    a.fixed = p->fixed;
    a.row_fix = p->row_fix;
    a.fix_sat = p->fix_sat;
    a.nu = sel<T>(p->nu64, p->nu32);
    a.offs = p->off_dev;
    a.br_row_ptr = p->n_pairs ? p->br_row_ptr : nullptr;
    a.br_node_i = p->br_node_i;
    a.br_bond_ptr = p->br_bond_ptr;
    a.br_q = p->br_q;
    a.br_off = p->br_off;
    a.ept = (a.rows + a.F - 1) / a.F;
    a.tl = a.ttx = a.tty = 0;
    a.treg = 0;
    a.tper = 1;
    a.tthreads = c.threads_tile;
    a.twt = nullptr;
    a.tspec = nullptr;
    a.tspecr = nullptr;
    a.tspec_slot = 0;
    a.stl = FftSched{};
    if (c.tile > 0 && p->dim == 2) {
        // frame spectra and twiddles exist for every configured tile length (built with the
        // configuration); an operator without them (the preconditioner's) runs the chain
        const TileSpec *ts = find_tile_spec(op, c.tile);
        const FftAxis *ta = find_tile_axis(p, c.tile);
        if (ts && ta) {
            const int inner = c.tile - 2 * p->M;
            a.tl = c.tile;
            a.ttx = (a.Nx + inner - 1) / inner;
            a.tty = (a.Ny + inner - 1) / inner;
            a.stl = make_sched(*ta, f32, c.max_radix);
            a.twt = tw_of<T>(*ta);
            a.tspec = sel<T>(ts->s64, ts->s32);
            a.tspecr = sel<T>(ts->r64, ts->r32);
            a.tspec_slot = multi ? (size_t)3 * c.tile * c.tile : 0;
            a.ept = a.ttx * a.tty;
            a.treg = c.tile_regs;
            a.tper = c.tile_regs ? c.tile_run : 1;
        }
    }
    return a;
}

template <typename K> static hipError_t allow_lds(K kern, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Launch geometry of one plan's chain: tiles per case of each pass, threads per block
// and dynamic LDS of each kernel.
struct ChainGeom {
    int tiles_x, tiles_l, tiles_y;   // x passes, line product (2D y / 3D z), 3D y passes
    int bx, bxi, bl;                 // threads: x-forward, x-inverse, line passes
    size_t lds_x, lds_l, lds_y;
};

template <typename T> static ChainGeom chain_geom(const PassArgs<T> &a) {
    const size_t cb = sizeof(cplx_t<T>);
    ChainGeom g;
    g.tiles_x = (a.rows + a.F - 1) / a.F;
    const int nzc = (a.Nz + a.Fl - 1) / a.Fl;
    g.tiles_y = a.d == 3 ? a.H * nzc : 0;
    g.tiles_l = ((a.d == 2 ? a.H : a.H * a.Ly) + a.Fl - 1) / a.Fl;
    g.bx = a.wave_x ? 64 * ((waves_x(a.d, a.F) + a.spw - 1) / a.spw) : a.bthreads;
    g.bxi = a.wave_x ? 64 * ((waves_x(a.d, a.F) + a.spw_i - 1) / a.spw_i) : a.bthreads;
    g.bl = a.wave_l ? 64 * ((a.Fl + a.lpw - 1) / a.lpw) : a.bthreads_line;
    g.lds_x = lds_x_bytes(a.d, a.F, a.sx.L, cb, a.ip_x);
    g.lds_l = lds_line_bytes(a.d, a.Fl, a.d == 2 ? a.sy.L : a.sz.L, cb, a.ip_l);
    g.lds_y = a.d == 3 ? lds_line_bytes(a.d, a.Fl, a.sy.L, cb, a.ip_l) : 0;
    return g;
}

// reps > 1 (single plans, measurement only): every pass is launched reps times back to
// back between the events, so an event interval is reps kernel durations without the
// dispatch gaps of a lone launch.
template <typename T, bool BX, bool BL, int RM>
static msb_status launch_chain(const PassArgs<T> &a, const EndArgs<T> &e, const ChainGeom &g, hipStream_t st,
                               hipEvent_t *ev, const PassArgs<T> *dA, const EndArgs<T> *dE, const GroupGrid *gg,
                               int reps = 1) {
    int evi = 0;
    auto mark = [&]() -> hipError_t { return ev ? hipEventRecord(ev[evi++], st) : hipSuccess; };
    MSB_HIP((gg ? allow_lds(k_xfwd_group<T, BX, RM>, g.lds_x) : allow_lds(k_xfwd<T, BX, RM>, g.lds_x)));
    MSB_HIP((gg ? allow_lds(k_xinv_group<T, BX, RM>, g.lds_x) : allow_lds(k_xinv<T, BX, RM>, g.lds_x)));
    MSB_HIP(mark());
    if (gg) hipLaunchKernelGGL((k_xfwd_group<T, BX, RM>), dim3(gg->total_x), dim3(g.bx), g.lds_x, st, dA, dE, gg->start_x, gg->n);
    else
        for (int k = 0; k < reps; ++k)
            hipLaunchKernelGGL((k_xfwd<T, BX, RM>), dim3(a.B * g.tiles_x), dim3(g.bx), g.lds_x, st, a, e);
    MSB_HIP(mark());
    if (a.d == 2) {
        MSB_HIP((gg ? allow_lds(k_line_y_group<T, BL, RM>, g.lds_l) : allow_lds(k_line_y<T, BL, RM>, g.lds_l)));
        if (gg) hipLaunchKernelGGL((k_line_y_group<T, BL, RM>), dim3(gg->total_l), dim3(g.bl), g.lds_l, st, dA, dE, gg->start_l, gg->n);
        else
            for (int k = 0; k < reps; ++k)
                hipLaunchKernelGGL((k_line_y<T, BL, RM>), dim3(a.B * g.tiles_l), dim3(g.bl), g.lds_l, st, a, e);
        MSB_HIP(mark());
    } else {
        MSB_HIP((gg ? allow_lds(k_yfwd_group<T, BL, RM>, g.lds_y) : allow_lds(k_yfwd<T, BL, RM>, g.lds_y)));
        MSB_HIP((gg ? allow_lds(k_yinv_group<T, BL, RM>, g.lds_y) : allow_lds(k_yinv<T, BL, RM>, g.lds_y)));
        MSB_HIP((gg ? allow_lds(k_line_z_group<T, BL, RM>, g.lds_l) : allow_lds(k_line_z<T, BL, RM>, g.lds_l)));
        if (gg) hipLaunchKernelGGL((k_yfwd_group<T, BL, RM>), dim3(gg->total_y), dim3(g.bl), g.lds_y, st, dA, dE, gg->start_y, gg->n);
        else
            for (int k = 0; k < reps; ++k)
                hipLaunchKernelGGL((k_yfwd<T, BL, RM>), dim3(a.B * g.tiles_y), dim3(g.bl), g.lds_y, st, a, e);
        MSB_HIP(mark());
        if (gg) hipLaunchKernelGGL((k_line_z_group<T, BL, RM>), dim3(gg->total_l), dim3(g.bl), g.lds_l, st, dA, dE, gg->start_l, gg->n);
        else
            for (int k = 0; k < reps; ++k)
                hipLaunchKernelGGL((k_line_z<T, BL, RM>), dim3(a.B * g.tiles_l), dim3(g.bl), g.lds_l, st, a, e);
        MSB_HIP(mark());
        if (gg) hipLaunchKernelGGL((k_yinv_group<T, BL, RM>), dim3(gg->total_y), dim3(g.bl), g.lds_y, st, dA, dE, gg->start_y, gg->n);
        else
            for (int k = 0; k < reps; ++k)
                hipLaunchKernelGGL((k_yinv<T, BL, RM>), dim3(a.B * g.tiles_y), dim3(g.bl), g.lds_y, st, a, e);
        MSB_HIP(mark());
    }
    if (gg) hipLaunchKernelGGL((k_xinv_group<T, BX, RM>), dim3(gg->total_x), dim3(g.bxi), g.lds_x, st, dA, dE, gg->start_x, gg->n);
    else
        for (int k = 0; k < reps; ++k)
            hipLaunchKernelGGL((k_xinv<T, BX, RM>), dim3(a.B * g.tiles_x), dim3(g.bxi), g.lds_x, st, a, e);
    MSB_HIP(mark());
    MSB_HIP(hipGetLastError());
    return MSB_OK;
}

// kernels built with RMAX = 8 only contain the basic radices 2, 3, 4, 5, 8
static bool needs_composite(const FftSched *const (&scheds)[3]) {
    for (const FftSched *sc : scheds)
        for (int i = 0; i < sc->np; ++i) {
            const int r = sc->ps[i].R;
            if (!(r == 2 || r == 3 || r == 4 || r == 5 || r == 8)) return true;
        }
    return false;
}

// Tiled product: a fused prologue first runs alone as the chain's x-forward kernel
// without its transform (it updates the vector the patches then read, and writes the
// solver's partial sums and flags; the patches overlap, so no tile may update in place),
// then one launch of the tile kernel over B x ttx x tty tiles.  ev (optional, 2 events)
// brackets the tile kernel; reps > 1 repeats it (measurement only).
template <typename T, bool BX>
static void launch_prologue(const PassArgs<T> &a, const EndArgs<T> &e, hipStream_t st) {
    EndArgs<T> ep = e;
    ep.no_transform = 1;
    const int bx = a.wave_x ? 64 * ((waves_x(a.d, a.F) + a.spw - 1) / a.spw) : a.bthreads;
    const int tiles_x = (a.rows + a.F - 1) / a.F;
    hipLaunchKernelGGL((k_xfwd<T, BX, 8>), dim3(a.B * tiles_x), dim3(bx), 0, st, a, ep);
}

template <typename T>
static msb_status launch_tiled(const PassArgs<T> &a, const EndArgs<T> &e, hipStream_t st, hipEvent_t *ev, int reps) {
    const size_t lds = lds_tile_bytes(a.tl, sizeof(cplx_t<T>));
    const FftSched *const sc[3] = {&a.stl, &a.stl, &a.stl};
    const bool comp = needs_composite(sc);
    if (e.pro != PRO_NONE) {
        if (a.wave_x) launch_prologue<T, false>(a, e, st);
        else launch_prologue<T, true>(a, e, st);
    }
    if (ev) MSB_HIP(hipEventRecord(ev[0], st));
    MSB_HIP(launch_tile_kernel<T>(a, e, lds, comp, reps, st));
    if (ev) MSB_HIP(hipEventRecord(ev[1], st));
    MSB_HIP(hipGetLastError());
    return MSB_OK;
}

template <typename T>
static msb_status dispatch_chain(const PassArgs<T> &a, const EndArgs<T> &e, const ChainGeom &g, bool composite,
                                 hipStream_t st, hipEvent_t *ev, const PassArgs<T> *dA, const EndArgs<T> *dE,
                                 const GroupGrid *gg, int reps = 1) {
    const int sel = (a.wave_x ? 1 : 0) | (a.wave_l ? 2 : 0) | (composite ? 4 : 0);
    switch (sel) {
        case 0: return launch_chain<T, true, true, 8>(a, e, g, st, ev, dA, dE, gg, reps);
        case 1: return launch_chain<T, false, true, 8>(a, e, g, st, ev, dA, dE, gg, reps);
        case 2: return launch_chain<T, true, false, 8>(a, e, g, st, ev, dA, dE, gg, reps);
        case 3: return launch_chain<T, false, false, 8>(a, e, g, st, ev, dA, dE, gg, reps);
        case 4: return launch_chain<T, true, true, 16>(a, e, g, st, ev, dA, dE, gg, reps);
        case 5: return launch_chain<T, false, true, 16>(a, e, g, st, ev, dA, dE, gg, reps);
        case 6: return launch_chain<T, true, false, 16>(a, e, g, st, ev, dA, dE, gg, reps);
        default: return launch_chain<T, false, false, 16>(a, e, g, st, ev, dA, dE, gg, reps);
    }
}

template <typename T>
msb_status launch_product(const PassArgs<T> &a, const EndArgs<T> &e, hipStream_t st, hipEvent_t *ev, int reps) {
    if (a.tl > 0 && a.corr) return launch_tiled<T>(a, e, st, ev, reps);
    const FftSched *const sc[3] = {&a.sx, &a.sy, &a.sz};
    return dispatch_chain<T>(a, e, chain_geom(a), needs_composite(sc), st, ev, nullptr, nullptr, nullptr, reps);
}

template <typename T>
msb_status launch_group(const PassArgs<T> &a, const GroupGrid &gg, const PassArgs<T> *dA, const EndArgs<T> *dE,
                        bool composite, hipStream_t st) {
    if (gg.tiled) {
        // a solver prologue first, as the transform-free x pass over the members' rows (the
        // members' end arguments carry no_transform), then the tiled kernel
        if (gg.pro) {
            const int bx = a.wave_x ? 64 * ((waves_x(a.d, a.F) + a.spw - 1) / a.spw) : a.bthreads;
            if (a.wave_x)
                hipLaunchKernelGGL((k_xfwd_group<T, false, 8>), dim3(gg.total_x), dim3(bx), 0, st, dA, dE, gg.start_x, gg.n);
            else
                hipLaunchKernelGGL((k_xfwd_group<T, true, 8>), dim3(gg.total_x), dim3(bx), 0, st, dA, dE, gg.start_x, gg.n);
        }
        const FftSched *const sc[3] = {&a.stl, &a.stl, &a.stl};
        MSB_HIP(launch_tile_group<T>(a, gg, dA, dE, needs_composite(sc), st));
        return MSB_OK;
    }
    ChainGeom g = chain_geom(a);
    g.lds_x = gg.lds_x;
    g.lds_l = gg.lds_l;
    g.lds_y = gg.lds_y;
    EndArgs<T> e;
    memset(&e, 0, sizeof(e));
    return dispatch_chain<T>(a, e, g, composite, st, nullptr, dA, dE, &gg);
}

void pass_tiles(const msb_plan_s *p, const msb_launch_config &c, bool fp32, int tiles[4], size_t lds[4]) {
    const size_t cb = fp32 ? sizeof(float2) : sizeof(double2);
    const int d = p->dim;
    const int H = (int)p->H, Ly = (int)p->L[1], Lz = (int)p->L[2], Nz = (int)p->n[2];
    tiles[0] = (int)((rows_total(p) + c.rows_per_wg - 1) / c.rows_per_wg);
    tiles[1] = ((d == 2 ? H : H * Ly) + c.lines_per_wg - 1) / c.lines_per_wg;
    tiles[2] = d == 3 ? H * ((Nz + c.lines_per_wg - 1) / c.lines_per_wg) : 0;
    lds[0] = lds_x_bytes(d, c.rows_per_wg, p->L[0], cb, c.lds_inplace & 1);
    lds[1] = lds_line_bytes(d, c.lines_per_wg, d == 2 ? Ly : Lz, cb, c.lds_inplace & 2);
    lds[2] = d == 3 ? lds_line_bytes(d, c.lines_per_wg, Ly, cb, c.lds_inplace & 2) : 0;
    tiles[3] = d == 2 ? tile_count(p, c.tile) : 0;
    lds[3] = d == 2 && c.tile > 0 ? (c.tile_regs ? 2 * (size_t)c.tile * (c.tile + 1) * cb : lds_tile_bytes(c.tile, cb)) : 0;
}

bool plan_needs_composite(const msb_plan_s *p, bool fp32, int max_radix) {
    const FftSched s0 = make_sched(p->ax[0], fp32, max_radix), s1 = make_sched(p->ax[1], fp32, max_radix),
                   s2 = make_sched(p->ax[2], fp32, max_radix);
    const FftSched *const sc[3] = {&s0, &s1, &s2};
    return needs_composite(sc);
}

template PassArgs<double> pass_args<double>(const msb_plan_s *, const DeviceOp &, const msb_launch_config *);
template PassArgs<float> pass_args<float>(const msb_plan_s *, const DeviceOp &, const msb_launch_config *);
template msb_status launch_product<double>(const PassArgs<double> &, const EndArgs<double> &, hipStream_t, hipEvent_t *,
                                          int);
template msb_status launch_product<float>(const PassArgs<float> &, const EndArgs<float> &, hipStream_t, hipEvent_t *,
                                         int);
template msb_status launch_group<double>(const PassArgs<double> &, const GroupGrid &, const PassArgs<double> *,
                                         const EndArgs<double> *, bool, hipStream_t);
template msb_status launch_group<float>(const PassArgs<float> &, const GroupGrid &, const PassArgs<float> *,
                                        const EndArgs<float> *, bool, hipStream_t);

}  // namespace msb
