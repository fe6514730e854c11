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
#include "fft_device.hpp"
#include "passes.hpp"

namespace msb {

constexpr int kThreads = 256;

__device__ __forceinline__ int comp_of(int a, int b, int d) {
    if (d == 2) return a + b;   // xx=0 xy=1 yy=2
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);   // xx xy xz yy yz zz
}

// ---------------------------------------------------------------------------- x-forward
template <typename T>
__global__ __launch_bounds__(kThreads) void k_xfwd(PassArgs<T> a, EndArgs<T> e) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[80];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int tpc = (a.rows + a.F - 1) / a.F;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int b = tile / tpc;
    const int r0 = (tile - b * tpc) * a.F;
    const int nr = min(a.F, a.rows - r0);
    const int nsig = a.d * nr;
    const int S = (nsig + 1) >> 1;
    const int Lx = a.sx.L;
    const int Smax = (a.d * a.F + 1) >> 1;
    T2 *bufA = reinterpret_cast<T2 *>(smem);
    T2 *bufB = bufA + (size_t)Smax * Lx;
    if (e.case_done && e.case_done[b]) return;

    T beta = T(0);
    if (e.pro == PRO_CG_P) {
        // r.r of the current residual decides convergence (flag 1) or a
        // non-finite residual (flag 3) before any work; beta = r.r / r_old.r_old
        const double rn = block_sum_partials(e.beta_part + (size_t)b * e.nbeta, e.nbeta, red, tid, nt);
        if (e.thresh && !(rn > e.thresh[b])) {
            if (r0 == 0 && tid == 0) e.done_rw[b] = (rn == rn && rn <= 1e300) ? 1 : 3;
            return;
        }
        if (e.beta_part_old) {
            const double ro = block_sum_partials(e.beta_part_old + (size_t)b * e.nbeta, e.nbeta, red, tid, nt);
            beta = ro > 0.0 ? T(rn / ro) : T(0);
        }
    }
    const T hdt2 = T(0.5 * e.dt * e.dt);
    const T dtt = T(e.dt);
    const size_t cbase = (size_t)b * a.d * a.N;

    for (int idx = tid; idx < S * Lx; idx += nt) {
        const int s = idx / Lx;
        const int n = idx - s * Lx;
        T2 z;
        z.x = T(0);
        z.y = T(0);
        if (n < a.Nx) {
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const int sig = 2 * s + h2;
                if (sig >= nsig) break;
                const int c = sig / nr;
                const int r = sig - c * nr;
                const int node = (r0 + r) * a.Nx + n;
                const size_t addr = cbase + (size_t)c * a.N + node;
                T v;
                if (e.pro == PRO_NONE) {
                    v = e.pio[addr];
                } else if (e.pro == PRO_CG_P) {
                    v = e.pr[addr] + beta * e.pio[addr];
                    e.pio[addr] = v;
                } else {
                    const bool fx = a.fixed && a.fixed[(size_t)c * a.N + node];
                    if (fx) v = e.pg ? e.pg[addr] : T(0);
                    else v = e.pio[addr] + dtt * e.pr[addr] + hdt2 * e.pa[addr];
                    e.pio[addr] = v;
                }
                if (h2 == 0) z.x = v;
                else z.y = v;
            }
        }
        bufA[idx] = z;
    }
    __syncthreads();
    T2 *res = fft_lds<T, T2, -1>(bufA, bufB, S, a.sx, a.twx, tid, nt);

    // unpack the two real transforms of each complex one; x-spectrum k < H
    for (int idx = tid; idx < nsig * a.H; idx += nt) {
        const int kx = idx / nsig;
        const int sig = idx - kx * nsig;
        const int s = sig >> 1;
        const T2 Z = res[s * Lx + kx];
        const T2 Zm = res[s * Lx + (kx == 0 ? 0 : Lx - kx)];
        T2 X;
        if ((sig & 1) == 0) {
            X.x = T(0.5) * (Z.x + Zm.x);
            X.y = T(0.5) * (Z.y - Zm.y);
        } else {
            X.x = T(0.5) * (Z.y + Zm.y);
            X.y = T(0.5) * (Zm.x - Z.x);
        }
        const int c = sig / nr;
        const int row = r0 + sig - c * nr;
        const int z = row / a.Ny;
        const int y = row - z * a.Ny;
        a.T1[((((size_t)b * a.d + c) * a.Nz + z) * a.H + kx) * a.Ny + y] = X;
    }
}

// ---------------------------------------------------------------------------- line product
// Lines of one case: data[((b*d + c)*nlines + line)*Nl + t], t < Nl.  Each line is
// zero-padded to L, transformed, multiplied by the real symmetric d x d spectrum
// block (spec[(comp*nlines + line)*L + k]) and transformed back.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_line_prod(PassArgs<T> a, EndArgs<T> e,
                                                       cplx_t<T> *data, int nlines, int Nl,
                                                       FftSched sl, const cplx_t<T> *twl) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int tpc = (nlines + a.Fl - 1) / a.Fl;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int b = tile / tpc;
    const int l0 = (tile - b * tpc) * a.Fl;
    const int nl = min(a.Fl, nlines - l0);
    const int d = a.d;
    const int S = nl * d;
    const int L = sl.L;
    T2 *bufA = reinterpret_cast<T2 *>(smem);
    T2 *bufB = bufA + (size_t)a.Fl * d * L;
    if (e.case_done && e.case_done[b]) return;

    for (int idx = tid; idx < S * L; idx += nt) {
        const int s = idx / L;
        const int t = idx - s * L;
        const int li = s / d;
        const int c = s - li * d;
        T2 v;
        v.x = T(0);
        v.y = T(0);
        if (t < Nl) v = data[(((size_t)b * d + c) * nlines + l0 + li) * Nl + t];
        bufA[idx] = v;
    }
    __syncthreads();
    T2 *res = fft_lds<T, T2, -1>(bufA, bufB, S, sl, twl, tid, nt);
    T2 *oth = (res == bufA) ? bufB : bufA;

    const T *spec = a.spec + (size_t)b * a.spec_slot;
    const size_t cstride = (size_t)nlines * L;
    for (int idx = tid; idx < nl * L; idx += nt) {
        const int li = idx / L;
        const int k = idx - li * L;
        const size_t g0 = (size_t)(l0 + li) * L + k;
        T2 *u = res + (size_t)li * d * L + k;
        if (d == 2) {
            const T gxx = spec[g0], gxy = spec[cstride + g0], gyy = spec[2 * cstride + g0];
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
            for (int q = 0; q < 6; ++q) g[q] = spec[q * cstride + g0];
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
    __syncthreads();
    T2 *out = fft_lds<T, T2, 1>(res, oth, S, sl, twl, tid, nt);
    for (int idx = tid; idx < S * Nl; idx += nt) {
        const int s = idx / Nl;
        const int t = idx - s * Nl;
        const int li = s / d;
        const int c = s - li * d;
        data[(((size_t)b * d + c) * nlines + l0 + li) * Nl + t] = out[(size_t)s * L + t];
    }
}

// ---------------------------------------------------------------------------- 3D y passes
// y-forward: T1[b][c][z][kx][y<Ny] -> T2[b][c][kx][ky<Ly][z], Fl z-planes per block.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_yfwd(PassArgs<T> a, EndArgs<T> e) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int d = a.d, Ly = a.sy.L;
    const int nzc = (a.Nz + a.Fl - 1) / a.Fl;
    const int tpc = a.H * nzc;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int b = tile / tpc;
    const int rem = tile - b * tpc;
    const int kx = rem / nzc;
    const int z0 = (rem - kx * nzc) * a.Fl;
    const int nz = min(a.Fl, a.Nz - z0);
    const int S = nz * d;
    T2 *bufA = reinterpret_cast<T2 *>(smem);
    T2 *bufB = bufA + (size_t)a.Fl * d * Ly;
    if (e.case_done && e.case_done[b]) return;
    for (int idx = tid; idx < S * Ly; idx += nt) {
        const int s = idx / Ly;
        const int t = idx - s * Ly;
        const int zl = s / d;
        const int c = s - zl * d;
        T2 v;
        v.x = T(0);
        v.y = T(0);
        if (t < a.Ny) v = a.T1[((((size_t)b * d + c) * a.Nz + z0 + zl) * a.H + kx) * a.Ny + t];
        bufA[idx] = v;
    }
    __syncthreads();
    T2 *res = fft_lds<T, T2, -1>(bufA, bufB, S, a.sy, a.twy, tid, nt);
    for (int idx = tid; idx < S * Ly; idx += nt) {
        const int zl = idx % nz;
        const int rest = idx / nz;
        const int c = rest % d;
        const int ky = rest / d;
        a.T2[((((size_t)b * d + c) * a.H + kx) * Ly + ky) * a.Nz + z0 + zl] = res[(zl * d + c) * Ly + ky];
    }
}

// y-inverse: T2[b][c][kx][ky][z] -> T1[b][c][z][kx][y<Ny]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_yinv(PassArgs<T> a, EndArgs<T> e) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int d = a.d, Ly = a.sy.L;
    const int nzc = (a.Nz + a.Fl - 1) / a.Fl;
    const int tpc = a.H * nzc;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int b = tile / tpc;
    const int rem = tile - b * tpc;
    const int kx = rem / nzc;
    const int z0 = (rem - kx * nzc) * a.Fl;
    const int nz = min(a.Fl, a.Nz - z0);
    const int S = nz * d;
    T2 *bufA = reinterpret_cast<T2 *>(smem);
    T2 *bufB = bufA + (size_t)a.Fl * d * Ly;
    if (e.case_done && e.case_done[b]) return;
    for (int idx = tid; idx < S * Ly; idx += nt) {
        const int zl = idx % nz;
        const int rest = idx / nz;
        const int c = rest % d;
        const int ky = rest / d;
        bufA[(zl * d + c) * Ly + ky] = a.T2[((((size_t)b * d + c) * a.H + kx) * Ly + ky) * a.Nz + z0 + zl];
    }
    __syncthreads();
    T2 *res = fft_lds<T, T2, 1>(bufA, bufB, S, a.sy, a.twy, tid, nt);
    for (int idx = tid; idx < S * a.Ny; idx += nt) {
        const int s = idx / a.Ny;
        const int t = idx - s * a.Ny;
        const int zl = s / d;
        const int c = s - zl * d;
        a.T1[((((size_t)b * d + c) * a.Nz + z0 + zl) * a.H + kx) * a.Ny + t] = res[(size_t)s * Ly + t];
    }
}

// ---------------------------------------------------------------------------- x-inverse
template <typename T>
__global__ __launch_bounds__(kThreads) void k_xinv(PassArgs<T> a, EndArgs<T> e) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[80];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int tpc = (a.rows + a.F - 1) / a.F;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int b = tile / tpc;
    const int r0 = (tile - b * tpc) * a.F;
    const int nr = min(a.F, a.rows - r0);
    const int d = a.d;
    const int nsig = d * nr;
    const int S = (nsig + 1) >> 1;
    const int Lx = a.sx.L;
    const int Smax = (d * a.F + 1) >> 1;
    T2 *bufA = reinterpret_cast<T2 *>(smem);
    T2 *bufB = bufA + (size_t)Smax * Lx;
    if (e.case_done && e.case_done[b]) return;

    // rebuild the full x-spectra of two real rows as one complex spectrum
    for (int idx = tid; idx < S * a.H; idx += nt) {
        const int kx = idx / S;
        const int s = idx - kx * S;
        T2 Xa, Xb;
        Xb.x = T(0);
        Xb.y = T(0);
        {
            const int sig = 2 * s, c = sig / nr, row = r0 + sig - c * nr;
            const int z = row / a.Ny, y = row - z * a.Ny;
            Xa = a.T1[((((size_t)b * d + c) * a.Nz + z) * a.H + kx) * a.Ny + y];
        }
        if (2 * s + 1 < nsig) {
            const int sig = 2 * s + 1, c = sig / nr, row = r0 + sig - c * nr;
            const int z = row / a.Ny, y = row - z * a.Ny;
            Xb = a.T1[((((size_t)b * d + c) * a.Nz + z) * a.H + kx) * a.Ny + y];
        }
        T2 Z;
        Z.x = Xa.x - Xb.y;
        Z.y = Xa.y + Xb.x;
        bufA[s * Lx + kx] = Z;
        const int m = Lx - kx;
        if (kx >= 1 && m >= a.H) {
            T2 Zm;
            Zm.x = Xa.x + Xb.y;
            Zm.y = -Xa.y + Xb.x;
            bufA[s * Lx + m] = Zm;
        }
    }
    __syncthreads();
    T2 *R = fft_lds<T, T2, 1>(bufA, bufB, S, a.sx, a.twx, tid, nt);
    T *Rr = reinterpret_cast<T *>(R);   // real output sig at Rr[2*((sig>>1)*Lx + n) + (sig&1)]

    const size_t cbase = (size_t)b * d * a.N;
    const T *uin = e.uin;

    // broken bonds (eq. (tea:fr)): f_p += sum_{q in v_p} W(q - p) (u_p - u_q)
    if (a.br_row_ptr) {
        const int e0 = a.br_row_ptr[r0], e1 = a.br_row_ptr[r0 + nr];
        const T *w = a.w + (size_t)b * a.w_slot;
        for (int idx = tid; idx < (e1 - e0) * d; idx += nt) {
            const int ei = e0 + idx / d;
            const int c = idx - (idx / d) * d;
            const int node = a.br_node_i[ei];
            const int row = node / a.Nx;
            const int n = node - row * a.Nx;
            double acc = 0.0;
            for (int t = a.br_bond_ptr[ei]; t < a.br_bond_ptr[ei + 1]; ++t) {
                const int q = a.br_q[t];
                const int o = a.br_off[t];
                for (int cb = 0; cb < d; ++cb) {
                    const double du = (double)uin[cbase + (size_t)cb * a.N + node] -
                                      (double)uin[cbase + (size_t)cb * a.N + q];
                    acc += (double)w[(size_t)comp_of(c, cb, d) * a.n_off + o] * du;
                }
            }
            const int sig = c * nr + (row - r0);
            Rr[2 * ((sig >> 1) * Lx + n) + (sig & 1)] += T(acc);
        }
        __syncthreads();
    }

    const T *de = a.de + (size_t)b * a.de_slot;
    const int M = a.M, M1 = a.M + 1;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    const T dth = T(0.5 * e.dt);
    const T rinv = T(1.0 / e.rho);
    for (int idx = tid; idx < nsig * a.Nx; idx += nt) {
        const int sig = idx / a.Nx;
        const int n = idx - sig * a.Nx;
        const int c = sig / nr;
        const int row = r0 + sig - c * nr;
        const int node = row * a.Nx + n;
        const size_t addr = cbase + (size_t)c * a.N + node;
        T f = Rr[2 * ((sig >> 1) * Lx + n) + (sig & 1)];
        // incomplete horizon (eq. (tea:sc)): table by clamped distances to the faces
        {
            const int z = row / a.Ny, y = row - z * a.Ny;
            const int lx = min(n, M), hx = min(a.Nx - 1 - n, M);
            const int ly = min(y, M), hy = min(a.Ny - 1 - y, M);
            int didx = ((lx * M1 + hx) * M1 + ly) * M1 + hy;
            bool interior = (lx == M) & (hx == M) & (ly == M) & (hy == M);
            if (d == 3) {
                const int lz = min(z, M), hz = min(a.Nz - 1 - z, M);
                didx = (didx * M1 + lz) * M1 + hz;
                interior = interior & (lz == M) & (hz == M);
            }
            if (!interior) {
                for (int cb = 0; cb < d; ++cb)
                    f += de[(size_t)comp_of(c, cb, d) * a.de_stride + didx] *
                         uin[cbase + (size_t)cb * a.N + node];
            }
        }
        const bool fx = a.fixed && a.fixed[(size_t)c * a.N + node];
        switch (e.epi) {
            case EPI_APPLY:
                e.out[addr] = fx ? T(0) : T(e.sign) * f;
                break;
            case EPI_CG_Q: {
                const T q = fx ? T(0) : -f;
                e.out[addr] = q;
                acc0 += (double)uin[addr] * (double)q;
                break;
            }
            case EPI_RESID: {
                const T v = fx ? T(0) : e.rhs[addr] + f;
                e.out[addr] = v;
                acc0 += (double)v * (double)v;
                break;
            }
            case EPI_VV: {
                T an = T(0), vn = T(0);
                const T bb = e.rhs[addr];
                if (!fx) {
                    an = (f + bb) * rinv;
                    vn = e.ev[addr] + dth * (e.ea[addr] + an);
                    if (e.energy) {
                        const double uu = (double)uin[addr];
                        acc0 += uu * (double)f;
                        acc1 += (double)vn * (double)vn;
                        acc2 += (double)bb * uu;
                    }
                }
                e.ea[addr] = an;
                e.ev[addr] = vn;
                break;
            }
            default:  // EPI_DOT
                if (!fx) acc0 += (double)e.rhs[addr] * (double)f;
                break;
        }
    }
    if (e.part) {
        double v[3] = {acc0, acc1, acc2};
        block_sum<3>(v, red, tid, nt);
        if (tid == 0) {
            const size_t stride = (size_t)gridDim.x;
            e.part[tile] = v[0];
            e.part[stride + tile] = v[1];
            e.part[2 * stride + tile] = v[2];
        }
    }
}

// ---------------------------------------------------------------------------- host side
int x_tiles_per_case(const msb_plan_s *p, int F) { return (int)((rows_total(p) + F - 1) / F); }

static size_t lds_budget() {
    static size_t b = 0;
    if (!b) {
        const char *e = getenv("MSB_LDS_BUDGET");
        b = e ? (size_t)atol(e) : (size_t)64 * 1024;
    }
    return b;
}

int rows_per_wg_for(const msb_plan_s *p, size_t cbytes) {
    const char *env = getenv("MSB_ROWS_PER_WG");
    if (env) return std::max(1, atoi(env));
    int F = 8;
    while (F > 1 && (size_t)2 * ((p->dim * F + 1) / 2) * p->L[0] * cbytes > lds_budget()) F /= 2;
    return F;
}

static int lines_per_wg_for(const msb_plan_s *p, size_t cbytes, int L) {
    const char *env = getenv("MSB_LINES_PER_WG");
    if (env) return std::max(1, atoi(env));
    int F = 8;
    while (F > 1 && (size_t)2 * F * p->dim * L * cbytes > lds_budget()) F /= 2;
    return F;
}

template <typename T> static const T *sel(const double *a, const float *b);
template <> const double *sel<double>(const double *a, const float *) { return a; }
template <> const float *sel<float>(const double *, const float *b) { return b; }

template <typename T> PassArgs<T> pass_args(const msb_plan_s *p, const DeviceOp &op) {
    PassArgs<T> a;
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
    a.F = rows_per_wg_for(p, sizeof(cplx_t<T>));
    a.Fl = lines_per_wg_for(p, sizeof(cplx_t<T>), p->dim == 2 ? (int)p->L[1] : (int)std::max(p->L[1], p->L[2]));
    a.sx = sched_of(p->ax[0]);
    a.sy = sched_of(p->ax[1]);
    a.sz = sched_of(p->ax[2]);
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
    a.br_row_ptr = p->n_pairs ? p->br_row_ptr : nullptr;
    a.br_node_i = p->br_node_i;
    a.br_bond_ptr = p->br_bond_ptr;
    a.br_q = p->br_q;
    a.br_off = p->br_off;
    return a;
}

template <typename K> static hipError_t allow_lds(K kern, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T>
msb_status launch_product(const PassArgs<T> &a, const EndArgs<T> &e, hipStream_t st, hipEvent_t *ev) {
    using T2 = cplx_t<T>;
    int evi = 0;
    auto mark = [&]() -> hipError_t { return ev ? hipEventRecord(ev[evi++], st) : hipSuccess; };
    const int tpc = (a.rows + a.F - 1) / a.F;
    const size_t lds_x = (size_t)2 * ((a.d * a.F + 1) / 2) * a.sx.L * sizeof(T2);
    MSB_HIP(allow_lds(k_xfwd<T>, lds_x));
    MSB_HIP(allow_lds(k_xinv<T>, lds_x));
    MSB_HIP(mark());
    hipLaunchKernelGGL(k_xfwd<T>, dim3(a.B * tpc), dim3(kThreads), lds_x, st, a, e);
    MSB_HIP(mark());
    if (a.d == 2) {
        const int lpc = (a.H + a.Fl - 1) / a.Fl;
        const size_t lds = (size_t)2 * a.Fl * a.d * a.sy.L * sizeof(T2);
        MSB_HIP(allow_lds(k_line_prod<T>, lds));
        hipLaunchKernelGGL(k_line_prod<T>, dim3(a.B * lpc), dim3(kThreads), lds, st, a, e, a.T1,
                           a.H, a.Ny, a.sy, a.twy);
        MSB_HIP(mark());
    } else {
        const int nzc = (a.Nz + a.Fl - 1) / a.Fl;
        const size_t lds_y = (size_t)2 * a.Fl * a.d * a.sy.L * sizeof(T2);
        MSB_HIP(allow_lds(k_yfwd<T>, lds_y));
        MSB_HIP(allow_lds(k_yinv<T>, lds_y));
        hipLaunchKernelGGL(k_yfwd<T>, dim3(a.B * a.H * nzc), dim3(kThreads), lds_y, st, a, e);
        MSB_HIP(mark());
        const int nlines = a.H * a.Ly;
        const int lpc = (nlines + a.Fl - 1) / a.Fl;
        const size_t lds_z = (size_t)2 * a.Fl * a.d * a.sz.L * sizeof(T2);
        MSB_HIP(allow_lds(k_line_prod<T>, lds_z));
        hipLaunchKernelGGL(k_line_prod<T>, dim3(a.B * lpc), dim3(kThreads), lds_z, st, a, e, a.T2,
                           nlines, a.Nz, a.sz, a.twz);
        MSB_HIP(mark());
        hipLaunchKernelGGL(k_yinv<T>, dim3(a.B * a.H * nzc), dim3(kThreads), lds_y, st, a, e);
        MSB_HIP(mark());
    }
    hipLaunchKernelGGL(k_xinv<T>, dim3(a.B * tpc), dim3(kThreads), lds_x, st, a, e);
    MSB_HIP(mark());
    MSB_HIP(hipGetLastError());
    return MSB_OK;
}

template PassArgs<double> pass_args<double>(const msb_plan_s *, const DeviceOp &);
template PassArgs<float> pass_args<float>(const msb_plan_s *, const DeviceOp &);
template msb_status launch_product<double>(const PassArgs<double> &, const EndArgs<double> &, hipStream_t, hipEvent_t *);
template msb_status launch_product<float>(const PassArgs<float> &, const EndArgs<float> &, hipStream_t, hipEvent_t *);

}  // namespace msb
