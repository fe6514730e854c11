// The tiled single-pass 2D product: one launch computes f = A u = A_hat u + D^e u +
// D^f u on blocks of the grid, each from an LDS-resident patch of u (the overlap-save
// form of Alg. 3), with the corrections, the constraint mask and the fused solver
// epilogues applied before the one store of f.
#include "epilogue.hpp"
#include "fft_device.hpp"
#include "passes.hpp"

namespace msb {

// Overlap-save form of the Toeplitz product: A_hat u at node p is the correlation
// sum_o K(o) u(p + o) over |o_a| <= M, u = 0 outside the grid (the zero embedding of
// Sec. 3.3).  A block of T x T nodes (T = tl - 2M) therefore needs u only on that block
// grown by M on every side: a tl x tl patch.  Its cyclic product with the generating
// array wrapped to tl x tl (Alg. 3 on the patch) differs from the linear one only where
// the kernel wraps around, within M of the patch edge; the inner T x T outputs are exact.
//
// The two displacement components go into one complex signal z = u_x + i u_y.  With
// Z = FFT(z), Ux = (Z(k) + conj Z(-k)) / 2 and Uy = (Z(k) - conj Z(-k)) / 2i, and the real
// even spectra Gxx, Gxy, Gyy, the block product written back as one complex signal
// w = f_x + i f_y is
//     W(k) = (Gxx + Gyy)/2 Z(k) + ((Gxx - Gyy)/2 + i Gxy) conj Z(-k),
// so a patch costs one forward and one inverse complex 2D transform in LDS (rows, then
// columns; the inverse only for the T inner rows at the end).  Then D^f, the surface
// correction and D^e are added on the inner block in LDS, and the mask and fused
// epilogue write the outputs: u is read once (plus the halo, from L2) and f written once.
// D^f sum of one Omega_br node p (eq. (tea:fr)): fxa, fya += sum over its directed broken
// bonds (q, o) of v_pq W(o) (u_p - u_q), v_pq = (nu_p + nu_q) / 2 on surface-corrected rows
// (on_e) and 1 elsewhere.  The bonds are loaded U at a time so that their index, u and
// weight loads are in flight together; the sum runs in bond order (as one at a time).
template <typename T, int U = 4>
__device__ __forceinline__ void df_bond_sum(const PassArgs<T> &a, const T *__restrict__ uin, size_t cbase, int N,
                                            const T *__restrict__ wt, int ei, bool on_e, double nup, double px,
                                            double py, double &fxa, double &fya) {
    const int t1 = a.br_bond_ptr[ei + 1];
    for (int t0 = a.br_bond_ptr[ei]; t0 < t1; t0 += U) {
        int q[U], oi[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int t = min(t0 + j, t1 - 1);
            q[j] = a.br_q[t];
            oi[j] = a.br_off[t];
        }
        double qx[U], qy[U], w0[U], w1[U], w2[U], nq[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            qx[j] = (double)uin[cbase + q[j]];
            qy[j] = (double)uin[cbase + N + q[j]];
            w0[j] = (double)wt[oi[j]];
            w1[j] = (double)wt[a.n_off + oi[j]];
            w2[j] = (double)wt[2 * a.n_off + oi[j]];
            nq[j] = on_e ? (double)a.nu[q[j]] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (t0 + j < t1) {
                const double dx = px - qx[j], dy = py - qy[j];
                const double v = on_e ? 0.5 * (nup + nq[j]) : 1.0;
                fxa += v * (w0[j] * dx + w1[j] * dy);
                fya += v * (w1[j] * dx + w2[j] * dy);
            }
        }
    }
}

// The broken-bond entries (the Omega_br nodes of eq. (tea:fr)) of a block's inner nodes,
// columns [x0, x0 + nx) of rows [y0, y0 + ny).  The entries of those rows span the whole
// grid width, so they are scanned kScan per thread at a time (independent loads) and the
// block's own are listed in lst as (entry, node) pairs; returns their count to every thread.
// lst holds 2 nx ny ints, and no thread may still use its memory when the first one calls.
// Each entry is a distinct node, so the order of the list does not change per-entry sums.
template <typename T>
__device__ __forceinline__ int list_block_bonds(const PassArgs<T> &a, int x0, int nx, int y0, int ny, int *lst,
                                                int tid, int nt) {
    __shared__ int cnt;
    if (tid == 0) cnt = 0;
    __syncthreads();
    const int Nx = a.Nx;
    const int e0 = a.br_row_ptr[y0], e1 = a.br_row_ptr[y0 + ny];
    constexpr int kScan = 8;
    for (int base = e0; base < e1; base += kScan * nt) {
        int nd[kScan];
#pragma unroll
        for (int j = 0; j < kScan; ++j) {
            const int ei = base + j * nt + tid;
            nd[j] = ei < e1 ? a.br_node_i[ei] : -1;
        }
#pragma unroll
        for (int j = 0; j < kScan; ++j) {
            const int qx = nd[j] - (nd[j] / Nx) * Nx;
            if (nd[j] >= 0 && qx >= x0 && qx < x0 + nx) {
                const int k = atomicAdd(&cnt, 1);
                lst[2 * k] = base + j * nt + tid;
                lst[2 * k + 1] = nd[j];
            }
        }
    }
    __syncthreads();
    return cnt;
}

template <typename T, int RMAX>
__device__ __forceinline__ void tile_body(const PassArgs<T> &a, const EndArgs<T> &e, int tile, int ntiles) {
    using T2 = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[96];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int Lt = a.tl, M = a.M, Tt = Lt - 2 * M;
    const int P = Lt | 1;                      // odd row pitch: conflict-free row and column stages
    const int tpc = a.ttx * a.tty;
    const int b = tile / tpc;
    const int rem = tile - b * tpc;
    const int ty = rem / a.ttx, tx = rem - ty * a.ttx;
    const int x0 = tx * Tt, y0 = ty * Tt;      // first inner node of the block
    const int nx = min(Tt, a.Nx - x0), ny = min(Tt, a.Ny - y0);   // inner nodes inside the grid
    T2 *tw = reinterpret_cast<T2 *>(smem);
    T2 *bufA = tw + Lt;
    T2 *bufB = bufA + (size_t)Lt * P;
    if (e.case_done && e.case_done[b]) return;
    stage_twiddles(tw, a.twt, Lt, tid, nt);
    const int N = a.N, Nx = a.Nx, Ny = a.Ny;
    const size_t cbase = (size_t)b * 2 * N;
    const T *uin = e.uin;
    {
        // patch node (lx, ly) = grid node (x0 - M + lx, y0 - M + ly); consecutive threads on
        // consecutive lx (contiguous in u and in LDS)
        const uint32_t mL = 0xFFFFFFFFu / (uint32_t)Lt + 1u;
        const T *ux = uin + cbase, *uy = ux + N;
        for (int i = tid; i < Lt * Lt; i += nt) {
            const int ly = (int)fdiv((uint32_t)i, mL), lx = i - ly * Lt;
            const int gx = x0 - M + lx, gy = y0 - M + ly;
            T2 z;
            z.x = T(0);
            z.y = T(0);
            if (gx >= 0 && gx < Nx && gy >= 0 && gy < Ny) {
                const size_t q = (size_t)gy * Nx + gx;
                z.x = ux[q];
                z.y = uy[q];
            }
            bufA[ly * P + lx] = z;
        }
    }
    __syncthreads();
    // forward: rows (signals P apart, elements adjacent), then columns
    T2 *r = fft_lds_2d<T, T2, -1, RMAX>(bufA, bufB, Lt, P, 1, a.stl, tw, tid, nt);
    T2 *o = r == bufA ? bufB : bufA;
    r = fft_lds_2d<T, T2, -1, RMAX>(r, o, Lt, 1, P, a.stl, tw, tid, nt);
    o = r == bufA ? bufB : bufA;
    {
        const T *g = a.tspec + (size_t)b * a.tspec_slot;
        const size_t n2 = (size_t)Lt * Lt;
        const uint32_t mL = 0xFFFFFFFFu / (uint32_t)Lt + 1u;
        for (int i = tid; i < Lt * Lt; i += nt) {
            const int ky = (int)fdiv((uint32_t)i, mL), kx = i - ky * Lt;
            const int mky = ky ? Lt - ky : 0, mkx = kx ? Lt - kx : 0;
            const T2 Z = r[ky * P + kx], Zm = r[mky * P + mkx];
            const T ga = g[i], gr = g[n2 + i], gi = g[2 * n2 + i];
            T2 W;
            W.x = ga * Z.x + gr * Zm.x + gi * Zm.y;
            W.y = ga * Z.y + gi * Zm.x - gr * Zm.y;
            o[ky * P + kx] = W;
        }
    }
    __syncthreads();
    // inverse: columns, then only the inner rows M .. M + T - 1
    r = fft_lds_2d<T, T2, 1, RMAX>(o, r, Lt, 1, P, a.stl, tw, tid, nt);
    o = r == bufA ? bufB : bufA;
    r = fft_lds_2d<T, T2, 1, RMAX>(r + M * P, o + M * P, Tt, P, 1, a.stl, tw, tid, nt);
    T2 *res = r + M;   // r starts at patch row M: inner node (jx, jy) at res[jy * P + jx], f_x + i f_y
    const T *wt = a.w + (size_t)b * a.w_slot;
    // broken bonds (eq. (tea:fr)): the Omega_br nodes of the block's rows are contiguous in
    // the per-row lists; f_p += sum_q W(q - p) (u_p - u_q) (with the surface correction a
    // bond of an Omega_e row carries v_pq W)
    if (a.br_row_ptr && ny > 0) {
        // the block's entries listed in the frame that does not hold the result, then summed
        // one per thread
        T2 *fr = r - (size_t)M * P == bufA ? bufB : bufA;
        const int cnt = list_block_bonds(a, x0, nx, y0, ny, reinterpret_cast<int *>(fr), tid, nt);
        const int *lst = reinterpret_cast<const int *>(fr);
        for (int k = tid; k < cnt; k += nt) {
            const int ei = lst[2 * k], node = lst[2 * k + 1];
            const int gy = node / Nx, gx = node - gy * Nx;
            const bool on_e = a.nu && (gx < M || gx >= Nx - M || gy < M || gy >= Ny - M);
            const double nup = on_e ? (double)a.nu[node] : 0.0;
            const double upx = (double)uin[cbase + node], upy = (double)uin[cbase + N + node];
            double fxa = 0.0, fya = 0.0;
            df_bond_sum<T>(a, uin, cbase, N, wt, ei, on_e, nup, upx, upy, fxa, fya);
            T2 &f = res[(gy - y0) * P + (gx - x0)];
            f.x += T(fxa);
            f.y += T(fya);
        }
        __syncthreads();
    }
    // nodes within M of a face (Omega_e): the surface correction (Remark 3, eq. (scr)) and
    // the incomplete-horizon diagonal D^e (eq. (tea:sc), table by clamped face distances)
    const bool edge = x0 < M || x0 + nx > Nx - M || y0 < M || y0 + ny > Ny - M;
    if (edge) {
        const T *de = a.de + (size_t)b * a.de_slot;
        const int M1 = M + 1;
        const uint32_t mT = 0xFFFFFFFFu / (uint32_t)Tt + 1u;
        for (int i = tid; i < Tt * Tt; i += nt) {
            const int jy = (int)fdiv((uint32_t)i, mT), jx = i - jy * Tt;
            if (jx >= nx || jy >= ny) continue;
            const int gx = x0 + jx, gy = y0 + jy;
            const int lx = min(gx, M), hx = min(Nx - 1 - gx, M), ly = min(gy, M), hy = min(Ny - 1 - gy, M);
            if ((lx == M) & (hx == M) & (ly == M) & (hy == M)) continue;   // full horizon
            const int node = gy * Nx + gx;
            const T upx = uin[cbase + node], upy = uin[cbase + N + node];
            T2 &f = res[jy * P + jx];
            if (a.nu) {
                const double nup = (double)a.nu[node];
                double ax = 0.0, ay = 0.0;
                for (int oi = 0; oi < a.n_off; ++oi) {
                    const int ox = a.offs[3 * oi], oy = a.offs[3 * oi + 1];
                    const int xx = gx + ox, yy = gy + oy;
                    if (xx < 0 || xx >= Nx || yy < 0 || yy >= Ny) continue;
                    const int q = node + oy * Nx + ox;
                    const double dx = (double)uin[cbase + q] - (double)upx, dy = (double)uin[cbase + N + q] - (double)upy;
                    const double vm = 0.5 * (nup + (double)a.nu[q]) - 1.0;
                    ax += vm * ((double)wt[oi] * dx + (double)wt[a.n_off + oi] * dy);
                    ay += vm * ((double)wt[a.n_off + oi] * dx + (double)wt[2 * a.n_off + oi] * dy);
                }
                f.x += T(ax);
                f.y += T(ay);
            }
            const int dx = ((lx * M1 + hx) * M1 + ly) * M1 + hy;
            const T dxx = de[dx], dxy = de[a.de_stride + dx], dyy = de[2 * a.de_stride + dx];
            f.x += dxx * upx + dxy * upy;
            f.y += dxy * upx + dyy * upy;
        }
        __syncthreads();
    }
    // mask and fused epilogue: both components of a node in one thread
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    {
        const T dth = T(0.5 * e.dt);
        const T rinv = T(1.0 / e.rho);
        const T sign = T(e.sign);
        const uint32_t mT = 0xFFFFFFFFu / (uint32_t)Tt + 1u;
        for (int i = tid; i < Tt * Tt; i += nt) {
            const int jy = (int)fdiv((uint32_t)i, mT), jx = i - jy * Tt;
            if (jx >= nx || jy >= ny) continue;
            const size_t node = (size_t)(y0 + jy) * Nx + (x0 + jx);
            const T2 f = res[jy * P + jx];
            const size_t ax = cbase + node, ay = ax + N;
            const bool fxx = a.fixed && a.fixed[node], fxy = a.fixed && a.fixed[N + node];
            epilogue_at<T>(e, uin, ax, ax - cbase + (size_t)b * e.pa_stride, f.x, fxx, sign, rinv, dth, acc0, acc1,
                           acc2);
            epilogue_at<T>(e, uin, ay, ay - cbase + (size_t)b * e.pa_stride, f.y, fxy, sign, rinv, dth, acc0, acc1,
                           acc2);
        }
    }
    if (e.part) {
        double v[3] = {acc0, acc1, acc2};
        block_sum<3>(v, red, tid, nt);
        if (tid == 0) {
            const size_t stride = (size_t)ntiles;
            e.part[tile] = v[0];
            e.part[stride + tile] = v[1];
            e.part[2 * stride + tile] = v[2];
        }
    }
}

template <typename T, int RMAX>
__global__ __launch_bounds__(kMaxBlock) void k_tile(PassArgs<T> a, EndArgs<T> e) {
    tile_body<T, RMAX>(a, e, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}

// ---------------------------------------------------------------------------- register-resident frames
// The same product with the frame transforms held in registers.  A frame length
// TL = R S (16 = 4 x 4, 32 = 8 x 4, 64 = 8 x 8) is cut into two Stockham stages: a thread
// owns R points of one line at positions p + S i (i < R), which are exactly the inputs of
// the first stage's radix-R butterfly p; after one exchange through LDS the thread computes
// R / S radix-S butterflies of the second stage (twiddles w_TL^(j m), held in registers),
// whose outputs land again at positions p + S i.  A 2D transform is a column transform,
// a transpose through LDS and a row transform, so each 1D transform costs one LDS
// round trip instead of one per stage, and the radix-R/S butterflies use compile-time
// constants.  The workgroup has S TL threads: thread t owns line t mod TL, part t div TL.
//
//   load     : column layout, thread (c, p) holds u at patch (row p + S i, column c)
//   forward  : column transform, transpose, row transform -> Z(ky = line, kx = p + S i)
//   product  : Z(-k) through one exchange; W = (Gxx + Gyy)/2 Z + ((Gxx - Gyy)/2 + i Gxy) conj Z(-k)
//   inverse  : row transform, transpose, column transform -> f at (row p + S i, column c),
//              the positions whose u the thread loaded (D^e u computed at load time)
//
// Exchanges alternate between two LDS frames, so one barrier per exchange suffices: a
// frame is written again only two exchanges later, after every thread has passed the
// barrier that follows its last read.
// The CG-epilogue form of the register kernel (p and r preloaded during the inverse
// transforms; the fused CG steps) exists where its registers keep the plain form's waves per
// SIMD: every frame in FP32, frame 16 in FP64 (FP64 frame 32 would take 258 registers).
template <typename T, int TL> constexpr bool cgq_form() { return sizeof(T) == 4 || TL == 16; }

template <int TL> struct RegShape;
template <> struct RegShape<16> { static constexpr int R = 4, S = 4; };
template <> struct RegShape<32> { static constexpr int R = 8, S = 4; };
template <> struct RegShape<64> { static constexpr int R = 8, S = 8; };

template <typename T, int TL, int DIR>
struct RegLine {
    using T2 = cplx_t<T>;
    static constexpr int R = RegShape<TL>::R, S = RegShape<TL>::S, RA = R / S;
    // 1D transform of the thread's line: v holds positions p + S i; element q of the line
    // lives at buf[q * es] (buf already offset to the line).  tw[a][m] = w_TL^((p + S a) m)
    // for the forward direction (conjugated here for the inverse).
    __device__ __forceinline__ static void run(T2 (&v)[R], T2 *buf, int es, int p, const T2 (&tw)[RA][S]) {
        Dft<T, T2, R, DIR>::run(v);
#pragma unroll
        for (int m = 0; m < R; ++m) buf[(p * R + m) * es] = v[m];
        __syncthreads();
#pragma unroll
        for (int a = 0; a < RA; ++a) {
            const int j = p + S * a;
            T2 t[S];
#pragma unroll
            for (int m = 0; m < S; ++m) t[m] = buf[(j + R * m) * es];
#pragma unroll
            for (int m = 1; m < S; ++m) {
                T2 w = tw[a][m];
                if (DIR > 0) w.y = -w.y;
                t[m] = c_mul(t[m], w);
            }
            Dft<T, T2, S, DIR>::run(t);
#pragma unroll
            for (int m = 0; m < S; ++m) v[a + RA * m] = t[m];
        }
    }
};

// One block per workgroup (tile_run = 1): every load of the block is issued at the start
// (spectra, u, constraint bits, D^e blocks), the D^e term is formed from u as it lands.
// CGQ: the CG epilogue (q = K p, partials p.q, r.q, q.q), whose p and r at the thread's
// output points are loaded before the inverse transforms so that the loads overlap them.
template <typename T, int TL, bool CGQ>
__device__ __forceinline__ void tile_reg_body(const PassArgs<T> &a, const EndArgs<T> &e, int tile, int ntiles) {
    using T2 = cplx_t<T>;
    constexpr int R = RegShape<TL>::R, S = RegShape<TL>::S, RA = R / S, P = TL + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[96];
    const int tid = threadIdx.x;
    const int ln = tid % TL, p = tid / TL;    // line and part
    const int M = a.M, Tt = TL - 2 * M;
    const int tpc = a.ttx * a.tty;
    const int b = tile / tpc;
    const int rem = tile - b * tpc;
    const int ty = rem / a.ttx, tx = rem - ty * a.ttx;
    const int x0 = tx * Tt, y0 = ty * Tt;      // first inner node of the block
    const int nx = min(Tt, a.Nx - x0), ny = min(Tt, a.Ny - y0);
    T2 *buf0 = reinterpret_cast<T2 *>(smem);
    T2 *buf1 = buf0 + TL * P;
    const int N = a.N, Nx = a.Nx, Ny = a.Ny;
    const size_t cbase = (size_t)b * 2 * N;
    const T *uin = e.uin;
    const bool edge = x0 < M || x0 + nx > Nx - M || y0 < M || y0 + ny > Ny - M;
    const int gx = x0 - M + ln;
    const bool col_in = gx >= 0 && gx < Nx;
    const bool col_inner = ln >= M && ln < M + nx;
    // fused CG step: alpha = r.r / p.q, the new r.r = r.r - 2 alpha r.q + alpha^2 q.q and
    // beta = new r.r / r.r from the case sums, with the stop and breakdown tests of the
    // prologue (one block per case writes the flags)
    const bool fused = CGQ && e.cg_fused == 1;
    const bool pfused = CGQ && e.cg_fused == 2;
    T alpha = T(0), beta = T(0);
    bool conv = false;
    if (pfused) {
        if (e.case_done[b]) {   // stopped: p of the inner nodes carried over to the new vector
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int ly = p + S * i;
                if (col_inner && ly >= M && ly < M + ny) {
                    const size_t ax = cbase + (size_t)(y0 - M + ly) * Nx + gx, ay = ax + N;
                    e.p_new[ax] = e.pio[ax];
                    e.p_new[ay] = e.pio[ay];
                }
            }
            return;
        }
        const double rz = e.case4[(size_t)b * 2], rzp = e.case4[(size_t)b * 2 + 1];
        beta = T(rzp > 0.0 ? rz / rzp : 0.0);
    } else if (fused) {
        const bool lead = rem == 0 && tid == 0;
        if (e.done_prev[b]) {
            // stopped before this step: carry the flag, and r, p of the inner nodes over to
            // the new vectors (every case's current vectors are then the new ones)
            if (lead) e.done_rw[b] = e.done_prev[b];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int ly = p + S * i;
                if (col_inner && ly >= M && ly < M + ny) {
                    const size_t ax = cbase + (size_t)(y0 - M + ly) * Nx + gx, ay = ax + N;
                    e.r_new[ax] = e.cr[ax];
                    e.r_new[ay] = e.cr[ay];
                    e.p_new[ax] = e.pio[ax];
                    e.p_new[ay] = e.pio[ay];
                }
            }
            return;
        }
        const double rr = e.case4[(size_t)b * 4], pq = e.case4[(size_t)b * 4 + 1];
        const double rq = e.case4[(size_t)b * 4 + 2], qq = e.case4[(size_t)b * 4 + 3];
        const double al = rr / pq;
        if (!(pq > 0.0) || !(al == al) || al > 1e300) {   // K not positive definite on p
            if (lead) e.done_rw[b] = 2;
            return;
        }
        const double rrn = rr - 2.0 * al * rq + al * al * qq;
        if (!(rrn == rrn)) {
            if (lead) e.done_rw[b] = 3;
            return;
        }
        alpha = T(al);
        beta = T(rr > 0.0 ? rrn / rr : 0.0);
        conv = e.update_only || (e.thresh && !(rrn > e.thresh[b]));
        if (lead) {
            e.iters[b] += 1;
            e.done_rw[b] = conv ? (e.update_only ? 5 : 1) : 0;
        }
    } else if (e.case_done && e.case_done[b]) {
        return;
    }
    // second-stage twiddles of this thread's butterflies (same in both axes)
    T2 tw[RA][S];
#pragma unroll
    for (int q = 0; q < RA; ++q)
#pragma unroll
        for (int m = 0; m < S; ++m) tw[q][m] = a.twt[(p + S * q) * m];
    // frame spectra of Z(ky = ln, kx = p + S i), stored in this thread order: register i of
    // all threads is one contiguous run
    const T *g = a.tspecr + (size_t)b * a.tspec_slot + tid;
    T ga[R], gr[R], gi[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        ga[i] = g[i * S * TL];
        gr[i] = g[TL * TL + i * S * TL];
        gi[i] = g[2 * TL * TL + i * S * TL];
    }
    // load: column layout, patch (row p + S i, column ln) = grid (x0 - M + ln, y0 - M + p + S i);
    // the D^e block of inner nodes within M of a face applied to u at load time, and the
    // constraint bits of the inner nodes.  Fused CG: u = p_new = r - alpha q + beta p from
    // the previous vectors at every patch node; the inner nodes' x, r, p updated.
    T2 v[R], dcor[R];
    T pux[R], puy[R], prx[R], pry[R];   // CG epilogue: p and r at the thread's inner nodes
    double rr_acc = 0.0;                // r.r of the inner nodes (fused step, rr_tiles)
    uint32_t fixbits = 0;
    const T *de = a.de + (size_t)b * a.de_slot;
    // constrained DOFs among the block's inner nodes, from the summed-area table of the mask:
    // without any, the block reads no mask.  Frames 32 and 64 only: their launches run in several
    // rounds of blocks, which hide the table's load; frame-16 blocks (one wave each, typically
    // all resident at once) wait for it at the start, which cost more than the mask loads saved
    // (one-case 512^2 FP32 product 6.4 -> 6.8 us; 16 cases at frame 32: 12% faster)
    bool bfix = a.fixed != nullptr;
    if (TL >= 32 && bfix && a.fix_sat) {
        const int W = Nx + 1;
        const int32_t *st = a.fix_sat;
        bfix = st[(y0 + ny) * W + x0 + nx] - st[y0 * W + x0 + nx] - st[(y0 + ny) * W + x0] + st[y0 * W + x0] > 0;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int ly = p + S * i, gy = y0 - M + ly;
        v[i].x = T(0);
        v[i].y = T(0);
        dcor[i].x = T(0);
        dcor[i].y = T(0);
        if (CGQ) pux[i] = puy[i] = prx[i] = pry[i] = T(0);
        if (col_in && gy >= 0 && gy < Ny) {
            const size_t q = (size_t)gy * Nx + gx;
            if (pfused) {   // p = z + beta p (the prologue's arithmetic)
                const size_t ax = cbase + q, ay = ax + N;
                v[i].x = e.pr[ax] + beta * e.pio[ax];
                v[i].y = e.pr[ay] + beta * e.pio[ay];
                if (col_inner && ly >= M && ly < M + ny) {
                    e.p_new[ax] = v[i].x;
                    e.p_new[ay] = v[i].y;
                }
            } else if (fused) {
                const size_t ax = cbase + q, ay = ax + N;
                const T px = e.pio[ax], py = e.pio[ay];
                const T rx = e.cr[ax] - alpha * e.cq[ax], ry = e.cr[ay] - alpha * e.cq[ay];
                v[i].x = rx + beta * px;
                v[i].y = ry + beta * py;
                if (col_inner && ly >= M && ly < M + ny) {
                    e.cx[ax] += alpha * px;
                    e.cx[ay] += alpha * py;
                    e.r_new[ax] = rx;
                    e.r_new[ay] = ry;
                    // a converged case keeps its last search direction (continuation)
                    e.p_new[ax] = conv ? px : v[i].x;
                    e.p_new[ay] = conv ? py : v[i].y;
                    rr_acc += (double)rx * (double)rx;
                    rr_acc += (double)ry * (double)ry;
                }
            } else {
                v[i].x = uin[cbase + q];
                v[i].y = uin[cbase + N + q];
            }
            if (col_inner && ly >= M && ly < M + ny) {
                if (bfix) fixbits |= ((uint32_t)a.fixed[q] | ((uint32_t)a.fixed[N + q] << 1)) << (2 * i);
                if (edge) {
                    const int M1 = M + 1;
                    const int lx = min(gx, M), hx = min(Nx - 1 - gx, M), lo = min(gy, M), hy = min(Ny - 1 - gy, M);
                    if (!((lx == M) & (hx == M) & (lo == M) & (hy == M))) {
                        const int di = ((lx * M1 + hx) * M1 + lo) * M1 + hy;
                        const T dxx = de[di], dxy = de[a.de_stride + di], dyy = de[2 * a.de_stride + di];
                        dcor[i].x = dxx * v[i].x + dxy * v[i].y;
                        dcor[i].y = dxy * v[i].x + dyy * v[i].y;
                    }
                }
            }
        }
    }
    if (fused && conv) {   // the final update only: no product
        double vs[1] = {rr_acc};
        block_sum<1>(vs, red, tid, S * TL);
        if (tid == 0) e.rr_out[tile] = vs[0];
        return;
    }
    // forward: columns (line ln, element q at buf[q P + ln]), transpose, rows
    RegLine<T, TL, -1>::run(v, buf0 + ln, P, p, tw);
#pragma unroll
    for (int i = 0; i < R; ++i) buf1[(p + S * i) * P + ln] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = buf1[ln * P + p + S * i];
    RegLine<T, TL, -1>::run(v, buf0 + ln * P, 1, p, tw);
    // block product with Z(-k) from the other frame
#pragma unroll
    for (int i = 0; i < R; ++i) buf1[ln * P + p + S * i] = v[i];
    __syncthreads();
    {
        const int mky = ln ? TL - ln : 0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int kx = p + S * i, mkx = kx ? TL - kx : 0;
            const T2 Z = v[i], Zm = buf1[mky * P + mkx];
            T2 W;
            W.x = ga[i] * Z.x + gr[i] * Zm.x + gi[i] * Zm.y;
            W.y = ga[i] * Z.y + gi[i] * Zm.x - gr[i] * Zm.y;
            v[i] = W;
        }
    }
    // CG epilogue: p (= u) and r at the output points, loaded now (in flight during the inverse);
    // fused: the new p and r this thread stored at those points in the load phase
    if (CGQ) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int ly = p + S * i;
            if (col_inner && ly >= M && ly < M + ny) {
                const size_t node = (size_t)(y0 - M + ly) * Nx + gx;
                pux[i] = uin[cbase + node];
                puy[i] = uin[cbase + N + node];
                prx[i] = e.rhs[cbase + node];
                pry[i] = e.rhs[cbase + N + node];
            }
        }
    }
    // inverse: rows, transpose, columns
    RegLine<T, TL, 1>::run(v, buf0 + ln * P, 1, p, tw);
#pragma unroll
    for (int i = 0; i < R; ++i) buf1[ln * P + p + S * i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = buf1[(p + S * i) * P + ln];
    RegLine<T, TL, 1>::run(v, buf0 + ln, P, p, tw);
    // broken bonds (eq. (tea:fr)) and the surface correction (Remark 3, eq. (scr)) of the
    // inner nodes, gathered into the free frame (zeroed first) by the nodes' threads of
    // the generic form, then read back by the owners
    const bool bonds = a.br_row_ptr && ny > 0 && a.br_row_ptr[y0] < a.br_row_ptr[y0 + ny];
    const bool surf = a.nu && edge;
    if (bonds || surf) {
        const int nt = S * TL;
        T2 *cor = buf1;
        for (int i = tid; i < TL * P; i += nt) {
            cor[i].x = T(0);
            cor[i].y = T(0);
        }
        __syncthreads();
        const T *wt = a.w + (size_t)b * a.w_slot;
        if (bonds) {
            // the block's entries listed in the free frame buf0 (2 Tt^2 ints fit in its
            // TL (TL + 1) complex elements), then summed one entry per thread
            const int cnt = list_block_bonds(a, x0, nx, y0, ny, reinterpret_cast<int *>(buf0), tid, nt);
            const int *lst = reinterpret_cast<const int *>(buf0);
            for (int k = tid; k < cnt; k += nt) {
                const int ei = lst[2 * k], node = lst[2 * k + 1];
                const int qy = node / Nx, qx = node - qy * Nx;
                const bool on_e = a.nu && (qx < M || qx >= Nx - M || qy < M || qy >= Ny - M);
                const double nup = on_e ? (double)a.nu[node] : 0.0;
                const double px = (double)uin[cbase + node], py = (double)uin[cbase + N + node];
                double fxa = 0.0, fya = 0.0;
                df_bond_sum<T>(a, uin, cbase, N, wt, ei, on_e, nup, px, py, fxa, fya);
                T2 &c = cor[(qy - y0 + M) * P + (qx - x0 + M)];
                c.x += T(fxa);
                c.y += T(fya);
            }
        }
        __syncthreads();
        if (surf) {
            for (int i = tid; i < Tt * Tt; i += nt) {
                const int jy = i / Tt, jx = i - jy * Tt;
                if (jx >= nx || jy >= ny) continue;
                const int qx = x0 + jx, qy = y0 + jy;
                if (qx >= M && qx < Nx - M && qy >= M && qy < Ny - M) continue;
                const int node = qy * Nx + qx;
                const double px = (double)uin[cbase + node], py = (double)uin[cbase + N + node];
                const double nup = (double)a.nu[node];
                double ax = 0.0, ay = 0.0;
                for (int oi = 0; oi < a.n_off; ++oi) {
                    const int ox = a.offs[3 * oi], oy = a.offs[3 * oi + 1];
                    const int xx = qx + ox, yy = qy + oy;
                    if (xx < 0 || xx >= Nx || yy < 0 || yy >= Ny) continue;
                    const int q = node + oy * Nx + ox;
                    const double dx = (double)uin[cbase + q] - px, dy = (double)uin[cbase + N + q] - py;
                    const double vm = 0.5 * (nup + (double)a.nu[q]) - 1.0;
                    ax += vm * ((double)wt[oi] * dx + (double)wt[a.n_off + oi] * dy);
                    ay += vm * ((double)wt[a.n_off + oi] * dx + (double)wt[2 * a.n_off + oi] * dy);
                }
                T2 &c = cor[(jy + M) * P + (jx + M)];
                c.x += T(ax);
                c.y += T(ay);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const T2 c = cor[(p + S * i) * P + ln];
            v[i].x += c.x;
            v[i].y += c.y;
        }
    }
    // D^e, mask and fused epilogue of the inner nodes this thread holds
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    {
        const T dth = T(0.5 * e.dt);
        const T rinv = T(1.0 / e.rho);
        const T sign = T(e.sign);
        const size_t pb = (size_t)b * e.pa_stride;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int ly = p + S * i;
            if (col_inner && ly >= M && ly < M + ny) {
                const size_t node = (size_t)(y0 - M + ly) * Nx + gx;
                const T fx = v[i].x + dcor[i].x, fy = v[i].y + dcor[i].y;
                const size_t ax = cbase + node, ay = ax + N;
                if (CGQ) {
                    // EPI_CG_Q with the preloaded p and r (the same arithmetic as epilogue_at)
                    const T qx = (fixbits >> (2 * i)) & 1u ? T(0) : -fx;
                    const T qy = (fixbits >> (2 * i + 1)) & 1u ? T(0) : -fy;
                    e.out[ax] = qx;
                    acc0 += (double)pux[i] * (double)qx;
                    acc1 += (double)prx[i] * (double)qx;
                    acc2 += (double)qx * (double)qx;
                    e.out[ay] = qy;
                    acc0 += (double)puy[i] * (double)qy;
                    acc1 += (double)pry[i] * (double)qy;
                    acc2 += (double)qy * (double)qy;
                    if (e.rr_tiles) {   // r.r of r = rhs (unfused step followed by fused ones)
                        rr_acc += (double)prx[i] * (double)prx[i];
                        rr_acc += (double)pry[i] * (double)pry[i];
                    }
                } else {
                    epilogue_at<T>(e, uin, ax, node + pb, fx, (fixbits >> (2 * i)) & 1u, sign, rinv, dth, acc0,
                                   acc1, acc2);
                    epilogue_at<T>(e, uin, ay, N + node + pb, fy, (fixbits >> (2 * i + 1)) & 1u, sign, rinv, dth,
                                   acc0, acc1, acc2);
                }
            }
        }
    }
    if (CGQ && (fused || e.rr_tiles)) {
        double vs[4] = {acc0, acc1, acc2, rr_acc};
        block_sum<4>(vs, red, tid, S * TL);
        if (tid == 0) {
            const size_t stride = (size_t)ntiles;
            e.part[tile] = vs[0];
            e.part[stride + tile] = vs[1];
            e.part[2 * stride + tile] = vs[2];
            e.rr_out[tile] = vs[3];
        }
    } else if (e.part) {
        double vs[3] = {acc0, acc1, acc2};
        block_sum<3>(vs, red, tid, S * TL);
        if (tid == 0) {
            const size_t stride = (size_t)ntiles;
            e.part[tile] = vs[0];
            e.part[stride + tile] = vs[1];
            e.part[2 * stride + tile] = vs[2];
        }
    }
}

template <typename T, int TL, bool CGQ>
__global__ __launch_bounds__(RegShape<TL>::S * TL) void k_tile_reg1(PassArgs<T> a, EndArgs<T> e) {
    tile_reg_body<T, TL, CGQ>(a, e, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}

// What a thread holds of one tile between its loads and its transforms: u at its R
// patch points (column layout), the D^e table index of its inner points within M of a
// face (-1 elsewhere) and the constraint bits of its inner points.
template <typename T, int TL> struct RegTile {
    static constexpr int R = RegShape<TL>::R;
    cplx_t<T> v[R];
    int di[R];
    uint32_t fix;
};

// Geometry of tile `tile` of a launch: case, first inner node, inner nodes in the grid.
struct TileGeom {
    int b, x0, y0, nx, ny, edge;
};
template <typename T>
__device__ __forceinline__ TileGeom tile_geom(const PassArgs<T> &a, int tile, int Tt) {
    TileGeom g;
    const int tpc = a.ttx * a.tty;
    g.b = tile / tpc;
    const int rem = tile - g.b * tpc;
    const int ty = rem / a.ttx, tx = rem - ty * a.ttx;
    g.x0 = tx * Tt;
    g.y0 = ty * Tt;
    g.nx = min(Tt, a.Nx - g.x0);
    g.ny = min(Tt, a.Ny - g.y0);
    g.edge = (g.x0 < a.M || g.x0 + g.nx > a.Nx - a.M || g.y0 < a.M || g.y0 + g.ny > a.Ny - a.M) ? 1 : 0;
    return g;
}

// Issue the loads of one tile: u at the thread's patch points and the constraint bits of
// its inner points; the D^e table index of its inner points within M of a face.
template <typename T, int TL>
__device__ __forceinline__ void reg_tile_load(const PassArgs<T> &a, const EndArgs<T> &e, const TileGeom &g, int ln,
                                              int p, RegTile<T, TL> &rt) {
    constexpr int R = RegShape<TL>::R, S = RegShape<TL>::S;
    const int M = a.M, N = a.N, Nx = a.Nx, Ny = a.Ny, M1 = M + 1;
    const size_t cbase = (size_t)g.b * 2 * N;
    const T *uin = e.uin;
    const int gx = g.x0 - M + ln;
    const bool col_in = gx >= 0 && gx < Nx;
    const bool col_inner = ln >= M && ln < M + g.nx;
    rt.fix = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int ly = p + S * i, gy = g.y0 - M + ly;
        rt.v[i].x = T(0);
        rt.v[i].y = T(0);
        rt.di[i] = -1;
        if (col_in && gy >= 0 && gy < Ny) {
            const size_t q = (size_t)gy * Nx + gx;
            rt.v[i].x = uin[cbase + q];
            rt.v[i].y = uin[cbase + N + q];
            if (col_inner && ly >= M && ly < M + g.ny) {
                if (a.fixed) rt.fix |= ((uint32_t)a.fixed[q] | ((uint32_t)a.fixed[N + q] << 1)) << (2 * i);
                const int lx = min(gx, M), hx = min(Nx - 1 - gx, M), lo = min(gy, M), hy = min(Ny - 1 - gy, M);
                if (g.edge && !((lx == M) & (hx == M) & (lo == M) & (hy == M)))
                    rt.di[i] = ((lx * M1 + hx) * M1 + lo) * M1 + hy;
            }
        }
    }
}

// D^e u at the thread's inner points within M of a face (eq. (tea:sc); the table is
// small and cache-resident), formed from the loaded u before the transforms overwrite it.
template <typename T, int TL>
__device__ __forceinline__ void reg_tile_de(const PassArgs<T> &a, const TileGeom &g, const RegTile<T, TL> &rt,
                                            cplx_t<T> (&dcor)[RegShape<TL>::R]) {
    constexpr int R = RegShape<TL>::R;
    const T *de = a.de + (size_t)g.b * a.de_slot;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        dcor[i].x = T(0);
        dcor[i].y = T(0);
        if (g.edge && rt.di[i] >= 0) {
            const int di = rt.di[i];
            const T dxx = de[di], dxy = de[a.de_stride + di], dyy = de[2 * a.de_stride + di];
            dcor[i].x = dxx * rt.v[i].x + dxy * rt.v[i].y;
            dcor[i].y = dxy * rt.v[i].x + dyy * rt.v[i].y;
        }
    }
}

// Transforms, block product, corrections and epilogue of one loaded tile.
template <typename T, int TL>
__device__ __forceinline__ void reg_tile_process(const PassArgs<T> &a, const EndArgs<T> &e, const TileGeom &g,
                                                 int tile, int ntiles, int ln, int p,
                                                 const cplx_t<T> (&tw)[RegShape<TL>::R / RegShape<TL>::S]
                                                                      [RegShape<TL>::S],
                                                 const T (&ga)[RegShape<TL>::R], const T (&gr)[RegShape<TL>::R],
                                                 const T (&gi)[RegShape<TL>::R], RegTile<T, TL> &rt,
                                                 const cplx_t<T> (&dcor)[RegShape<TL>::R], cplx_t<T> *buf0,
                                                 cplx_t<T> *buf1, double *red) {
    using T2 = cplx_t<T>;
    constexpr int R = RegShape<TL>::R, S = RegShape<TL>::S, P = TL + 1;
    const int tid = threadIdx.x;
    const int M = a.M, Tt = TL - 2 * M;
    const int N = a.N, Nx = a.Nx, Ny = a.Ny;
    const size_t cbase = (size_t)g.b * 2 * N;
    const T *uin = e.uin;
    T2(&v)[R] = rt.v;
    // forward: columns (line ln, element q at buf[q P + ln]), transpose, rows
    RegLine<T, TL, -1>::run(v, buf0 + ln, P, p, tw);
#pragma unroll
    for (int i = 0; i < R; ++i) buf1[(p + S * i) * P + ln] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = buf1[ln * P + p + S * i];
    RegLine<T, TL, -1>::run(v, buf0 + ln * P, 1, p, tw);
    // block product with Z(-k) from the other frame
#pragma unroll
    for (int i = 0; i < R; ++i) buf1[ln * P + p + S * i] = v[i];
    __syncthreads();
    {
        const int mky = ln ? TL - ln : 0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int kx = p + S * i, mkx = kx ? TL - kx : 0;
            const T2 Z = v[i], Zm = buf1[mky * P + mkx];
            T2 W;
            W.x = ga[i] * Z.x + gr[i] * Zm.x + gi[i] * Zm.y;
            W.y = ga[i] * Z.y + gi[i] * Zm.x - gr[i] * Zm.y;
            v[i] = W;
        }
    }
    // inverse: rows, transpose, columns
    RegLine<T, TL, 1>::run(v, buf0 + ln * P, 1, p, tw);
#pragma unroll
    for (int i = 0; i < R; ++i) buf1[ln * P + p + S * i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = buf1[(p + S * i) * P + ln];
    RegLine<T, TL, 1>::run(v, buf0 + ln, P, p, tw);
    // broken bonds (eq. (tea:fr)) and the surface correction (Remark 3, eq. (scr)) of the
    // inner nodes, gathered into the free frame (zeroed first), read back by the owners
    const bool bonds = a.br_row_ptr && g.ny > 0 && a.br_row_ptr[g.y0] < a.br_row_ptr[g.y0 + g.ny];
    const bool surf = a.nu && g.edge;
    if (bonds || surf) {
        const int nt = S * TL;
        T2 *cor = buf1;
        for (int i = tid; i < TL * P; i += nt) {
            cor[i].x = T(0);
            cor[i].y = T(0);
        }
        __syncthreads();
        const T *wt = a.w + (size_t)g.b * a.w_slot;
        if (bonds) {
            // the block's entries listed in the free frame buf0, then summed one per thread
            const int cnt = list_block_bonds(a, g.x0, g.nx, g.y0, g.ny, reinterpret_cast<int *>(buf0), tid, nt);
            const int *lst = reinterpret_cast<const int *>(buf0);
            for (int k = tid; k < cnt; k += nt) {
                const int ei = lst[2 * k], node = lst[2 * k + 1];
                const int qy = node / Nx, qx = node - qy * Nx;
                const bool on_e = a.nu && (qx < M || qx >= Nx - M || qy < M || qy >= Ny - M);
                const double nup = on_e ? (double)a.nu[node] : 0.0;
                const double px = (double)uin[cbase + node], py = (double)uin[cbase + N + node];
                double fxa = 0.0, fya = 0.0;
                df_bond_sum<T, 1>(a, uin, cbase, N, wt, ei, on_e, nup, px, py, fxa, fya);
                T2 &c = cor[(qy - g.y0 + M) * P + (qx - g.x0 + M)];
                c.x += T(fxa);
                c.y += T(fya);
            }
        }
        __syncthreads();
        if (surf) {
            for (int i = tid; i < Tt * Tt; i += nt) {
                const int jy = i / Tt, jx = i - jy * Tt;
                if (jx >= g.nx || jy >= g.ny) continue;
                const int qx = g.x0 + jx, qy = g.y0 + jy;
                if (qx >= M && qx < Nx - M && qy >= M && qy < Ny - M) continue;
                const int node = qy * Nx + qx;
                const double px = (double)uin[cbase + node], py = (double)uin[cbase + N + node];
                const double nup = (double)a.nu[node];
                double ax = 0.0, ay = 0.0;
                for (int oi = 0; oi < a.n_off; ++oi) {
                    const int ox = a.offs[3 * oi], oy = a.offs[3 * oi + 1];
                    const int xx = qx + ox, yy = qy + oy;
                    if (xx < 0 || xx >= Nx || yy < 0 || yy >= Ny) continue;
                    const int q = node + oy * Nx + ox;
                    const double dx = (double)uin[cbase + q] - px, dy = (double)uin[cbase + N + q] - py;
                    const double vm = 0.5 * (nup + (double)a.nu[q]) - 1.0;
                    ax += vm * ((double)wt[oi] * dx + (double)wt[a.n_off + oi] * dy);
                    ay += vm * ((double)wt[a.n_off + oi] * dx + (double)wt[2 * a.n_off + oi] * dy);
                }
                T2 &c = cor[(jy + M) * P + (jx + M)];
                c.x += T(ax);
                c.y += T(ay);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const T2 c = cor[(p + S * i) * P + ln];
            v[i].x += c.x;
            v[i].y += c.y;
        }
        // the frame is written again by the next tile's first exchange
        __syncthreads();
    }
    // D^e, mask and fused epilogue of the inner nodes this thread holds
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    {
        const T dth = T(0.5 * e.dt);
        const T rinv = T(1.0 / e.rho);
        const T sign = T(e.sign);
        const size_t pb = (size_t)g.b * e.pa_stride;
        const int gx = g.x0 - M + ln;
        const bool col_inner = ln >= M && ln < M + g.nx;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int ly = p + S * i;
            if (col_inner && ly >= M && ly < M + g.ny) {
                const size_t node = (size_t)(g.y0 - M + ly) * Nx + gx;
                const T fx = v[i].x + dcor[i].x, fy = v[i].y + dcor[i].y;
                const size_t ax = cbase + node, ay = ax + N;
                if (e.epi == EPI_APPLY) {
                    const T ox = (rt.fix >> (2 * i)) & 1u ? T(0) : sign * fx;
                    const T oy = (rt.fix >> (2 * i + 1)) & 1u ? T(0) : sign * fy;
                    if (e.wt) {
                        st_wt(&e.out[ax], ox);
                        st_wt(&e.out[ay], oy);
                    } else {
                        e.out[ax] = ox;
                        e.out[ay] = oy;
                    }
                } else {
                    epilogue_at<T>(e, uin, ax, node + pb, fx, (rt.fix >> (2 * i)) & 1u, sign, rinv, dth, acc0, acc1,
                                   acc2);
                    epilogue_at<T>(e, uin, ay, N + node + pb, fy, (rt.fix >> (2 * i + 1)) & 1u, sign, rinv, dth,
                                   acc0, acc1, acc2);
                }
            }
        }
    }
    if (e.part) {
        double vs[3] = {acc0, acc1, acc2};
        block_sum<3>(vs, red, tid, S * TL);
        if (tid == 0) {
            const size_t stride = (size_t)ntiles;
            e.part[tile] = vs[0];
            e.part[stride + tile] = vs[1];
            e.part[2 * stride + tile] = vs[2];
        }
    }
}

// Runs (tile_run > 1): a workgroup processes the a.tper consecutive tiles [first, first + tper) of
// the launch's ntiles (XCD-remapped runs, so that neighbouring blocks, whose patches
// overlap, share an L2): the loads of the next tile are issued before the transforms of
// the current one, so memory and arithmetic of consecutive tiles overlap.
template <typename T, int TL>
__device__ __forceinline__ void tile_reg_run(const PassArgs<T> &a, const EndArgs<T> &e, int run, int ntiles) {
    using T2 = cplx_t<T>;
    constexpr int R = RegShape<TL>::R, S = RegShape<TL>::S, RA = R / S, P = TL + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[96];
    const int tid = threadIdx.x;
    const int ln = tid % TL, p = tid / TL;    // line and part
    const int Tt = TL - 2 * a.M;
    T2 *buf0 = reinterpret_cast<T2 *>(smem);
    T2 *buf1 = buf0 + TL * P;
    const int first = run * a.tper, last = min(first + a.tper, ntiles);
    // second-stage twiddles of this thread's butterflies (same in both axes and every tile)
    T2 tw[RA][S];
#pragma unroll
    for (int q = 0; q < RA; ++q)
#pragma unroll
        for (int m = 0; m < S; ++m) tw[q][m] = a.twt[(p + S * q) * m];
    // frame spectra of Z(ky = ln, kx = p + S i): per case slot (reloaded when the case changes)
    T ga[R], gr[R], gi[R];
    int gb = -1;
    RegTile<T, TL> cur, nxt;
    TileGeom g = tile_geom(a, first, Tt);
    if (first < last) reg_tile_load<T, TL>(a, e, g, ln, p, cur);
    for (int t = first; t < last; ++t) {
        TileGeom gn = g;
        if (t + 1 < last) {
            gn = tile_geom(a, t + 1, Tt);
            reg_tile_load<T, TL>(a, e, gn, ln, p, nxt);
        }
        if (!(e.case_done && e.case_done[g.b])) {
            const int slot = a.tspec_slot ? g.b : 0;
            if (slot != gb) {
                const T *gs = a.tspecr + (size_t)slot * a.tspec_slot + tid;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    ga[i] = gs[i * S * TL];
                    gr[i] = gs[TL * TL + i * S * TL];
                    gi[i] = gs[2 * TL * TL + i * S * TL];
                }
                gb = slot;
            }
            T2 dcor[R];
            reg_tile_de<T, TL>(a, g, cur, dcor);
            reg_tile_process<T, TL>(a, e, g, t, ntiles, ln, p, tw, ga, gr, gi, cur, dcor, buf0, buf1, red);
            // the next tile exchanges through the frames in the other order: its first
            // writes go to the frame this tile last read before its final barrier
            T2 *sw = buf0;
            buf0 = buf1;
            buf1 = sw;
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            cur.v[i] = nxt.v[i];
            cur.di[i] = nxt.di[i];
        }
        cur.fix = nxt.fix;
        g = gn;
    }
}

template <typename T, int TL>
__global__ __launch_bounds__(RegShape<TL>::S * TL) void k_tile_reg(PassArgs<T> a, EndArgs<T> e) {
    tile_reg_run<T, TL>(a, e, xcd_tile(blockIdx.x, gridDim.x), a.B * a.ttx * a.tty);
}

// ---------------------------------------------------------------------------- plan groups
// One launch over the blocks of several plans: each workgroup finds its member in start[]
// after the XCD remap and takes that member's arguments from the device arrays.

template <typename T, int RMAX>
__global__ __launch_bounds__(kMaxBlock) void k_tile_group(const PassArgs<T> *__restrict__ A,
                                                          const EndArgs<T> *__restrict__ E,
                                                          const int *__restrict__ start, int n) {
    const int g = xcd_tile(blockIdx.x, gridDim.x);
    const int m = group_member(start, n, g);
    tile_body<T, RMAX>(A[m], E[m], g - start[m], start[m + 1] - start[m]);
}

template <typename T, int TL, bool CGQ>
__global__ __launch_bounds__(RegShape<TL>::S * TL) void k_tile_reg1_group(const PassArgs<T> *__restrict__ A,
                                                                       const EndArgs<T> *__restrict__ E,
                                                                       const int *__restrict__ start, int n) {
    const int g = xcd_tile(blockIdx.x, gridDim.x);
    const int m = group_member(start, n, g);
    tile_reg_body<T, TL, CGQ>(A[m], E[m], g - start[m], start[m + 1] - start[m]);
}

template <typename K> static hipError_t allow_lds(K kern, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Largest plain-product output written through the L2s (a quarter of their 8 x 4 MB).
constexpr size_t kWtMaxBytes = 8u << 20;

// Register-frame launch for frame length TL: runs of blocks, the CG-epilogue form (frame 16,
// whose registers leave room for the preloaded p and r) or the plain one-block form.
template <typename T, int TL>
static hipError_t launch_reg(const PassArgs<T> &a, const EndArgs<T> &e, dim3 gridr, dim3 grid, size_t lr, int reps,
                             hipStream_t st) {
    hipError_t err;
    const dim3 block(RegShape<TL>::S * TL);
    if (a.tper > 1) {
        if ((err = allow_lds(k_tile_reg<T, TL>, lr)) != hipSuccess) return err;
        for (int k = 0; k < reps; ++k) hipLaunchKernelGGL((k_tile_reg<T, TL>), gridr, block, lr, st, a, e);
        return hipGetLastError();
    }
    if constexpr (cgq_form<T, TL>()) {
        if (e.epi == EPI_CG_Q) {
            if ((err = allow_lds(k_tile_reg1<T, TL, true>, lr)) != hipSuccess) return err;
            for (int k = 0; k < reps; ++k) hipLaunchKernelGGL((k_tile_reg1<T, TL, true>), grid, block, lr, st, a, e);
            return hipGetLastError();
        }
    }
    if ((err = allow_lds(k_tile_reg1<T, TL, false>, lr)) != hipSuccess) return err;
    for (int k = 0; k < reps; ++k) hipLaunchKernelGGL((k_tile_reg1<T, TL, false>), grid, block, lr, st, a, e);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tile_kernel(const PassArgs<T> &a, const EndArgs<T> &e0, size_t lds, bool composite, int reps,
                              hipStream_t st) {
    const dim3 grid(a.B * a.ttx * a.tty), block(a.tthreads);
    hipError_t err;
    // a plain product whose output is at most kWtMaxBytes is written through the L2s (st_wt)
    EndArgs<T> e = e0;
    e.wt = e.epi == EPI_APPLY && (size_t)a.B * 2 * a.N * sizeof(T) <= kWtMaxBytes;
    if (a.treg) {
        // register-resident frames: S TL threads, two TL x (TL + 1) frames
        const size_t lr = 2 * (size_t)a.tl * (a.tl + 1) * sizeof(cplx_t<T>);
        const int tiles = a.B * a.ttx * a.tty;
        const dim3 gridr((tiles + a.tper - 1) / a.tper);
        switch (a.tl) {
            case 16: return launch_reg<T, 16>(a, e, gridr, grid, lr, reps, st);
            case 32: return launch_reg<T, 32>(a, e, gridr, grid, lr, reps, st);
            case 64: return launch_reg<T, 64>(a, e, gridr, grid, lr, reps, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (composite) {
        if ((err = allow_lds(k_tile<T, 16>, lds)) != hipSuccess) return err;
        for (int k = 0; k < reps; ++k) hipLaunchKernelGGL((k_tile<T, 16>), grid, block, lds, st, a, e);
    } else {
        if ((err = allow_lds(k_tile<T, 8>, lds)) != hipSuccess) return err;
        for (int k = 0; k < reps; ++k) hipLaunchKernelGGL((k_tile<T, 8>), grid, block, lds, st, a, e);
    }
    return hipGetLastError();
}

template hipError_t launch_tile_kernel<double>(const PassArgs<double> &, const EndArgs<double> &, size_t, bool, int,
                                               hipStream_t);
template hipError_t launch_tile_kernel<float>(const PassArgs<float> &, const EndArgs<float> &, size_t, bool, int,
                                              hipStream_t);

}  // namespace msb

namespace msb {

template <typename T, int TL, bool CGQ>
static hipError_t launch_reg_group(const GroupGrid &gg, const PassArgs<T> *dA, const EndArgs<T> *dE, hipStream_t st) {
    const hipError_t err = allow_lds(k_tile_reg1_group<T, TL, CGQ>, gg.lds_t);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_tile_reg1_group<T, TL, CGQ>), dim3(gg.total_t), dim3(RegShape<TL>::S * TL), gg.lds_t, st, dA,
                       dE, gg.start_t, gg.n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tile_group(const PassArgs<T> &a, const GroupGrid &gg, const PassArgs<T> *dA, const EndArgs<T> *dE,
                             bool composite, hipStream_t st) {
    hipError_t err;
    const dim3 grid(gg.total_t);
    if (a.treg) {
        switch (a.tl) {
            // CG slots (epilogue q = K p) at frame 16: the form that preloads p and r
            case 16: return gg.cgq ? launch_reg_group<T, 16, true>(gg, dA, dE, st)
                                   : launch_reg_group<T, 16, false>(gg, dA, dE, st);
            case 32:
                if constexpr (cgq_form<T, 32>())
                    if (gg.cgq) return launch_reg_group<T, 32, true>(gg, dA, dE, st);
                return launch_reg_group<T, 32, false>(gg, dA, dE, st);
            case 64:
                if constexpr (cgq_form<T, 64>())
                    if (gg.cgq) return launch_reg_group<T, 64, true>(gg, dA, dE, st);
                return launch_reg_group<T, 64, false>(gg, dA, dE, st);
            default: return hipErrorInvalidValue;
        }
    } else if (composite) {
        if ((err = allow_lds(k_tile_group<T, 16>, gg.lds_t)) != hipSuccess) return err;
        hipLaunchKernelGGL((k_tile_group<T, 16>), grid, dim3(a.tthreads), gg.lds_t, st, dA, dE, gg.start_t, gg.n);
    } else {
        if ((err = allow_lds(k_tile_group<T, 8>, gg.lds_t)) != hipSuccess) return err;
        hipLaunchKernelGGL((k_tile_group<T, 8>), grid, dim3(a.tthreads), gg.lds_t, st, dA, dE, gg.start_t, gg.n);
    }
    return hipGetLastError();
}

template hipError_t launch_tile_group<double>(const PassArgs<double> &, const GroupGrid &, const PassArgs<double> *,
                                              const EndArgs<double> *, bool, hipStream_t);
template hipError_t launch_tile_group<float>(const PassArgs<float> &, const GroupGrid &, const PassArgs<float> *,
                                             const EndArgs<float> *, bool, hipStream_t);

}  // namespace msb
