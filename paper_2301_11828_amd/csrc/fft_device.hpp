// Device-side batched complex FFT in LDS: mixed-radix Stockham autosort passes
// (radices 2, 3, 4, 5, 8), ping-pong between two LDS buffers, natural order in and
// out.  Used by every pass of the FFT product (Alg. 3 / Alg. 4 of the paper
// evaluate the Toeplitz part A_hat u through FFT, Hadamard product, inverse FFT).
//
// Pass with radix R after Ns points have been combined (Ns = product of the
// radices of the earlier passes): butterfly j of a signal reads x[j + m L/R],
// m < R, twiddles input m by w^(k m) with w = exp(-2 pi i / (Ns R)), k = j mod Ns,
// applies the length-R DFT and writes y[(j div Ns) Ns R + k + m Ns].  The twiddle
// w^(k m) = exp(-2 pi i t / L) with t = k m L / (Ns R) < L is read from one table
// per length, computed on the host with exact angle reduction.
#pragma once

#include "common.hpp"

namespace msb {

template <typename T2> __device__ __forceinline__ T2 c_make(double x, double y) {
    T2 r;
    r.x = x;
    r.y = y;
    return r;
}

template <typename T2> __device__ __forceinline__ T2 c_add(T2 a, T2 b) {
    T2 r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename T2> __device__ __forceinline__ T2 c_sub(T2 a, T2 b) {
    T2 r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <typename T2> __device__ __forceinline__ T2 c_mul(T2 a, T2 b) {
    T2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// a * (s i), s = +1 or -1
template <typename T2> __device__ __forceinline__ T2 c_muli(T2 a, int s) {
    T2 r;
    r.x = -s * a.y;
    r.y = s * a.x;
    return r;
}
template <typename T2> __device__ __forceinline__ T2 c_conj(T2 a) {
    a.y = -a.y;
    return a;
}

// Length-R DFT in registers; DIR = -1 forward (exp(-2 pi i ms/R)), +1 inverse.
template <typename T, typename T2, int R, int DIR> struct Dft;

template <typename T, typename T2, int DIR> struct Dft<T, T2, 2, DIR> {
    __device__ __forceinline__ static void run(T2 *v, const T2 *__restrict__ tw = nullptr, int lr = 0) {
        T2 a = v[0], b = v[1];
        v[0] = c_add(a, b);
        v[1] = c_sub(a, b);
    }
};

template <typename T, typename T2, int DIR> struct Dft<T, T2, 3, DIR> {
    __device__ __forceinline__ static void run(T2 *v, const T2 *__restrict__ tw = nullptr, int lr = 0) {
        const T c = T(-0.5);
        const T s = T(DIR) * T(0.86602540378443864676372317075294);   // forward: -sin(2 pi/3)
        T2 t = c_add(v[1], v[2]);
        T2 d = c_sub(v[1], v[2]);
        T2 m;
        m.x = v[0].x + c * t.x;
        m.y = v[0].y + c * t.y;
        v[0] = c_add(v[0], t);
        // v1 = m + i s d ; v2 = m - i s d  (s carries the direction)
        T2 isd;
        isd.x = -s * d.y;
        isd.y = s * d.x;
        v[1] = c_add(m, isd);
        v[2] = c_sub(m, isd);
    }
};

template <typename T, typename T2, int DIR> struct Dft<T, T2, 4, DIR> {
    __device__ __forceinline__ static void run(T2 *v, const T2 *__restrict__ tw = nullptr, int lr = 0) {
        T2 t0 = c_add(v[0], v[2]);
        T2 t1 = c_sub(v[0], v[2]);
        T2 t2 = c_add(v[1], v[3]);
        T2 t3 = c_sub(v[1], v[3]);
        // forward: V1 = t1 - i t3, V3 = t1 + i t3
        T2 it3 = c_muli(t3, DIR);  // DIR * i * t3
        v[0] = c_add(t0, t2);
        v[2] = c_sub(t0, t2);
        v[1] = c_add(t1, it3);
        v[3] = c_sub(t1, it3);
    }
};

template <typename T, typename T2, int DIR> struct Dft<T, T2, 5, DIR> {
    __device__ __forceinline__ static void run(T2 *v, const T2 *__restrict__ tw = nullptr, int lr = 0) {
        const T c1 = T(0.30901699437494742410229341718282);    // cos(2 pi/5)
        const T c2 = T(-0.80901699437494742410229341718282);   // cos(4 pi/5)
        const T s1 = T(DIR) * T(0.95105651629515357211643933337938);   // forward: -sin(2 pi/5)
        const T s2 = T(DIR) * T(0.58778525229247312916870595463907);   // forward: -sin(4 pi/5)
        T2 t1 = c_add(v[1], v[4]);
        T2 t2 = c_add(v[2], v[3]);
        T2 d1 = c_sub(v[1], v[4]);
        T2 d2 = c_sub(v[2], v[3]);
        T2 a1, a2;
        a1.x = v[0].x + c1 * t1.x + c2 * t2.x;
        a1.y = v[0].y + c1 * t1.y + c2 * t2.y;
        a2.x = v[0].x + c2 * t1.x + c1 * t2.x;
        a2.y = v[0].y + c2 * t1.y + c1 * t2.y;
        // b1 = s1 d1 + s2 d2 ; b2 = s2 d1 - s1 d2 ; V1 = a1 + i b1, V4 = a1 - i b1,
        // V2 = a2 + i b2, V3 = a2 - i b2 (signs of s carry the direction)
        T2 b1, b2;
        b1.x = s1 * d1.x + s2 * d2.x;
        b1.y = s1 * d1.y + s2 * d2.y;
        b2.x = s2 * d1.x - s1 * d2.x;
        b2.y = s2 * d1.y - s1 * d2.y;
        v[0].x = v[0].x + t1.x + t2.x;
        v[0].y = v[0].y + t1.y + t2.y;
        v[1].x = a1.x - b1.y;
        v[1].y = a1.y + b1.x;
        v[4].x = a1.x + b1.y;
        v[4].y = a1.y - b1.x;
        v[2].x = a2.x - b2.y;
        v[2].y = a2.y + b2.x;
        v[3].x = a2.x + b2.y;
        v[3].y = a2.y - b2.x;
    }
};

template <typename T, typename T2, int DIR> struct Dft<T, T2, 8, DIR> {
    __device__ __forceinline__ static void run(T2 *v, const T2 *__restrict__ tw = nullptr, int lr = 0) {
        const T r = T(0.70710678118654752440084436210485);
        // two radix-4 DFTs on even and odd samples, then combine with w8^m
        T2 e[4] = {v[0], v[2], v[4], v[6]};
        T2 o[4] = {v[1], v[3], v[5], v[7]};
        Dft<T, T2, 4, DIR>::run(e, tw, lr);
        Dft<T, T2, 4, DIR>::run(o, tw, lr);
        // w8 = exp(DIR * 2 pi i / 8): w^1 = r(1 + DIR i), w^2 = DIR i, w^3 = r(-1 + DIR i)
        T2 o1, o2, o3;
        o1.x = r * (o[1].x - T(DIR) * o[1].y);
        o1.y = r * (o[1].y + T(DIR) * o[1].x);
        o2 = c_muli(o[2], DIR);
        o3.x = r * (-o[3].x - T(DIR) * o[3].y);
        o3.y = r * (-o[3].y + T(DIR) * o[3].x);
        v[0] = c_add(e[0], o[0]);
        v[4] = c_sub(e[0], o[0]);
        v[1] = c_add(e[1], o1);
        v[5] = c_sub(e[1], o1);
        v[2] = c_add(e[2], o2);
        v[6] = c_sub(e[2], o2);
        v[3] = c_add(e[3], o3);
        v[7] = c_sub(e[3], o3);
    }
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t m) { return m ? __umulhi(n, m) : n; }

// Division by a block-uniform divisor d < 2^16 for numerators n < 2^16 (exact);
// falls back to plain division when the numerator range is larger.
struct FastDiv {
    uint32_t d, m;
    bool exact;
    __device__ __forceinline__ FastDiv(uint32_t dd, uint32_t nmax) : d(dd) {
        exact = dd < 65536u && nmax < 65536u;
        m = dd <= 1 ? 0u : 0xFFFFFFFFu / dd + 1u;   // ceil(2^32 / d), 32-bit arithmetic
    }
    __device__ __forceinline__ uint32_t div(uint32_t n) const { return exact ? fdiv(n, m) : n / d; }
};

// Composite radix R = R1 * R2 (6, 9, 10, 12, 15, 16) computed in registers (two-level Cooley-Tukey):
// input index m = m1 + R1 m2, output index s = s2 + R2 s1;
//   A[m1][s2] = DFT_R2 over m2 of v[m1 + R1 m2];  A[m1][s2] *= W_R^(m1 s2);
//   V[s2 + R2 s1] = DFT_R1 over m1 of A[m1][s2].
// W_R^t = tw[t * lr] from the length-L table (lr = L / R), conjugated for DIR = +1.
template <typename T, typename T2, int R1, int R2, int DIR> struct Dft2 {
    __device__ __forceinline__ static void run(T2 *v, const T2 *__restrict__ tw, int lr) {
        T2 A[R1][R2];
#pragma unroll
        for (int m1 = 0; m1 < R1; ++m1) {
#pragma unroll
            for (int m2 = 0; m2 < R2; ++m2) A[m1][m2] = v[m1 + R1 * m2];
            Dft<T, T2, R2, DIR>::run(A[m1], tw, lr * R1);
        }
#pragma unroll
        for (int m1 = 1; m1 < R1; ++m1)
#pragma unroll
            for (int s2 = 1; s2 < R2; ++s2) {
                T2 w = tw[m1 * s2 * lr];
                if (DIR > 0) w.y = -w.y;
                A[m1][s2] = c_mul(A[m1][s2], w);
            }
#pragma unroll
        for (int s2 = 0; s2 < R2; ++s2) {
            T2 col[R1];
#pragma unroll
            for (int m1 = 0; m1 < R1; ++m1) col[m1] = A[m1][s2];
            Dft<T, T2, R1, DIR>::run(col, tw, lr * R2);
#pragma unroll
            for (int s1 = 0; s1 < R1; ++s1) v[s2 + R2 * s1] = col[s1];
        }
    }
};

#define MSB_COMPOSITE(R, R1, R2)                                                              \
    template <typename T, typename T2, int DIR> struct Dft<T, T2, R, DIR> {                   \
        __device__ __forceinline__ static void run(T2 *v, const T2 *__restrict__ tw, int lr) { \
            Dft2<T, T2, R1, R2, DIR>::run(v, tw, lr);                                         \
        }                                                                                     \
    };
MSB_COMPOSITE(6, 3, 2)
MSB_COMPOSITE(9, 3, 3)
MSB_COMPOSITE(10, 5, 2)
MSB_COMPOSITE(12, 4, 3)
MSB_COMPOSITE(15, 5, 3)
MSB_COMPOSITE(16, 4, 4)
#undef MSB_COMPOSITE

// One Stockham pass over S signals of length L stored back to back; twiddles in LDS.
template <typename T, typename T2, int R, int DIR>
__device__ __forceinline__ void stockham_pass(const T2 *__restrict__ in, T2 *__restrict__ out, int S,
                                              int L, const FftPass &ps, const T2 *__restrict__ tw,
                                              int tid, int nt) {
    const int nb = ps.nb;
    const int Ns = ps.Ns;
    const int total = S * nb;
    for (int t = tid; t < total; t += nt) {
        const int s = (int)fdiv((uint32_t)t, ps.m_nb);
        const int j = t - s * nb;
        const T2 *x = in + s * L;
        T2 v[R];
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = x[j + m * nb];
        const int jq = (int)fdiv((uint32_t)j, ps.m_Ns);
        const int k = j - jq * Ns;
        if (Ns > 1) {
            const int step = k * ps.twstep;
#pragma unroll
            for (int m = 1; m < R; ++m) {
                T2 w = tw[m * step];
                if (DIR > 0) w.y = -w.y;
                v[m] = c_mul(v[m], w);
            }
        }
        Dft<T, T2, R, DIR>::run(v, tw, L / R);
        T2 *y = out + s * L + jq * Ns * R + k;
#pragma unroll
        for (int m = 0; m < R; ++m) y[m * Ns] = v[m];
    }
}

// Ordering point between Stockham stages of signals owned by a single wavefront:
// LDS traffic of one wave is processed in order, so a wave-scope fence plus a
// scheduling barrier is all that is needed (no block-wide s_barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Butterflies of one in-place stage a thread may own: they stay in registers between
// the stage's reads and writes, at most as many values as one radix-RMAX butterfly.
__host__ __device__ constexpr int inplace_batch(int R, int RMAX) { return RMAX / R > 1 ? RMAX / R : 1; }

// The same stage in place: every thread reads and transforms all its butterflies (at
// most inplace_batch(R, RMAX) of them; the host checks S nb <= that many per thread),
// the team synchronises (BLOCK: workgroup barrier, else wave scope), then every
// thread writes its outputs into the buffer it read.
template <typename T, typename T2, int R, int DIR, int RMAX, bool BLOCK>
__device__ __forceinline__ void stockham_pass_ip(T2 *buf, int S, int L, const FftPass &ps,
                                                 const T2 *__restrict__ tw, int tid, int nt) {
    constexpr int KB = inplace_batch(R, RMAX);
    const int nb = ps.nb;
    const int Ns = ps.Ns;
    const int total = S * nb;
    T2 v[KB][R];
    int ob[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        const int t = tid + i * nt;
        ob[i] = -1;
        if (t < total) {
            const int s = (int)fdiv((uint32_t)t, ps.m_nb);
            const int j = t - s * nb;
            const T2 *x = buf + s * L;
#pragma unroll
            for (int m = 0; m < R; ++m) v[i][m] = x[j + m * nb];
            const int jq = (int)fdiv((uint32_t)j, ps.m_Ns);
            const int k = j - jq * Ns;
            if (Ns > 1) {
                const int step = k * ps.twstep;
#pragma unroll
                for (int m = 1; m < R; ++m) {
                    T2 w = tw[m * step];
                    if (DIR > 0) w.y = -w.y;
                    v[i][m] = c_mul(v[i][m], w);
                }
            }
            Dft<T, T2, R, DIR>::run(v[i], tw, L / R);
            ob[i] = s * L + jq * Ns * R + k;
        }
    }
    if (BLOCK) __syncthreads();
    else wave_sync();
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        if (ob[i] < 0) continue;
        T2 *y = buf + ob[i];
#pragma unroll
        for (int m = 0; m < R; ++m) y[m * Ns] = v[i][m];
    }
}

template <typename T, typename T2, int DIR, int RMAX, bool BLOCK>
__device__ void fft_inplace(T2 *a, int S, const FftSched &sc, const T2 *__restrict__ tw, int tid, int nt) {
    const int L = sc.L;
    for (int p = 0; p < sc.np; ++p) {
        const FftPass &ps = sc.ps[p];
        switch (ps.R) {
            case 2: stockham_pass_ip<T, T2, 2, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
            case 3: stockham_pass_ip<T, T2, 3, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
            case 4: stockham_pass_ip<T, T2, 4, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
            case 5: stockham_pass_ip<T, T2, 5, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
            case 8: stockham_pass_ip<T, T2, 8, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
            default:
                if constexpr (RMAX >= 16) {
                    switch (ps.R) {
                        case 6: stockham_pass_ip<T, T2, 6, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
                        case 9: stockham_pass_ip<T, T2, 9, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
                        case 10: stockham_pass_ip<T, T2, 10, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
                        case 12: stockham_pass_ip<T, T2, 12, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
                        case 15: stockham_pass_ip<T, T2, 15, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
                        default: stockham_pass_ip<T, T2, 16, DIR, RMAX, BLOCK>(a, S, L, ps, tw, tid, nt); break;
                    }
                }
                break;
        }
        if (BLOCK) __syncthreads();
        else wave_sync();
    }
}

// Full transform of S signals in LDS buffer a (scratch b); tw: the length-L twiddle
// table staged in LDS.  Returns the buffer that holds the result.  Every thread of
// the block must call it (it synchronises).
template <typename T, typename T2, int DIR, int RMAX>
__device__ T2 *fft_lds(T2 *a, T2 *b, int S, const FftSched &sc, const T2 *__restrict__ tw,
                       int tid, int nt) {
    const int L = sc.L;
    for (int p = 0; p < sc.np; ++p) {
        const FftPass &ps = sc.ps[p];
        switch (ps.R) {
            case 2: stockham_pass<T, T2, 2, DIR>(a, b, S, L, ps, tw, tid, nt); break;
            case 3: stockham_pass<T, T2, 3, DIR>(a, b, S, L, ps, tw, tid, nt); break;
            case 4: stockham_pass<T, T2, 4, DIR>(a, b, S, L, ps, tw, tid, nt); break;
            case 5: stockham_pass<T, T2, 5, DIR>(a, b, S, L, ps, tw, tid, nt); break;
            case 8: stockham_pass<T, T2, 8, DIR>(a, b, S, L, ps, tw, tid, nt); break;
            default:
                if constexpr (RMAX >= 16) {
                    switch (ps.R) {
                        case 6: stockham_pass<T, T2, 6, DIR>(a, b, S, L, ps, tw, tid, nt); break;
                        case 9: stockham_pass<T, T2, 9, DIR>(a, b, S, L, ps, tw, tid, nt); break;
                        case 10: stockham_pass<T, T2, 10, DIR>(a, b, S, L, ps, tw, tid, nt); break;
                        case 12: stockham_pass<T, T2, 12, DIR>(a, b, S, L, ps, tw, tid, nt); break;
                        case 15: stockham_pass<T, T2, 15, DIR>(a, b, S, L, ps, tw, tid, nt); break;
                        default: stockham_pass<T, T2, 16, DIR>(a, b, S, L, ps, tw, tid, nt); break;
                    }
                }
                break;
        }
        __syncthreads();
        T2 *t = a;
        a = b;
        b = t;
    }
    return a;
}

// Transform of S signals owned by one wavefront (lane = 0..63) in its private LDS
// buffers a/b; returns the buffer holding the result.  No block barrier.
template <typename T, typename T2, int DIR, int RMAX>
__device__ T2 *fft_wave(T2 *a, T2 *b, int S, const FftSched &sc, const T2 *__restrict__ tw, int lane) {
    const int L = sc.L;
    for (int p = 0; p < sc.np; ++p) {
        const FftPass &ps = sc.ps[p];
        switch (ps.R) {
            case 2: stockham_pass<T, T2, 2, DIR>(a, b, S, L, ps, tw, lane, 64); break;
            case 3: stockham_pass<T, T2, 3, DIR>(a, b, S, L, ps, tw, lane, 64); break;
            case 4: stockham_pass<T, T2, 4, DIR>(a, b, S, L, ps, tw, lane, 64); break;
            case 5: stockham_pass<T, T2, 5, DIR>(a, b, S, L, ps, tw, lane, 64); break;
            case 8: stockham_pass<T, T2, 8, DIR>(a, b, S, L, ps, tw, lane, 64); break;
            default:
                if constexpr (RMAX >= 16) {
                    switch (ps.R) {
                        case 6: stockham_pass<T, T2, 6, DIR>(a, b, S, L, ps, tw, lane, 64); break;
                        case 9: stockham_pass<T, T2, 9, DIR>(a, b, S, L, ps, tw, lane, 64); break;
                        case 10: stockham_pass<T, T2, 10, DIR>(a, b, S, L, ps, tw, lane, 64); break;
                        case 12: stockham_pass<T, T2, 12, DIR>(a, b, S, L, ps, tw, lane, 64); break;
                        case 15: stockham_pass<T, T2, 15, DIR>(a, b, S, L, ps, tw, lane, 64); break;
                        default: stockham_pass<T, T2, 16, DIR>(a, b, S, L, ps, tw, lane, 64); break;
                    }
                }
                break;
        }
        wave_sync();
        T2 *t = a;
        a = b;
        b = t;
    }
    return a;
}

// One Stockham stage over S signals of length L held in a 2D LDS array: element m of
// signal s at s * ss + m * es (rows of a frame: ss = row pitch, es = 1; columns: ss = 1,
// es = row pitch).  Consecutive threads take the same butterfly of consecutive signals,
// so with an odd row pitch a wavefront's accesses fall on distinct LDS banks in both
// directions.  mS = ceil(2^32 / S) (0 for S = 1).
template <typename T, typename T2, int R, int DIR>
__device__ __forceinline__ void stockham_pass_2d(const T2 *__restrict__ in, T2 *__restrict__ out, int S, uint32_t mS,
                                                 int L, int ss, int es, const FftPass &ps,
                                                 const T2 *__restrict__ tw, int tid, int nt) {
    const int nb = ps.nb;
    const int Ns = ps.Ns;
    const int total = S * nb;
    for (int t = tid; t < total; t += nt) {
        const int j = (int)fdiv((uint32_t)t, mS);
        const int s = t - j * S;
        const T2 *x = in + s * ss + j * es;
        T2 v[R];
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = x[m * nb * es];
        const int jq = (int)fdiv((uint32_t)j, ps.m_Ns);
        const int k = j - jq * Ns;
        if (Ns > 1) {
            const int step = k * ps.twstep;
#pragma unroll
            for (int m = 1; m < R; ++m) {
                T2 w = tw[m * step];
                if (DIR > 0) w.y = -w.y;
                v[m] = c_mul(v[m], w);
            }
        }
        Dft<T, T2, R, DIR>::run(v, tw, L / R);
        T2 *y = out + s * ss + (jq * Ns * R + k) * es;
#pragma unroll
        for (int m = 0; m < R; ++m) y[m * Ns * es] = v[m];
    }
}

// All stages of the length-L transform of S signals of a 2D LDS array (layout as for
// stockham_pass_2d), ping-pong between a and b with a block barrier after each stage;
// returns the buffer that holds the result.  Every thread of the block must call it.
template <typename T, typename T2, int DIR, int RMAX>
__device__ T2 *fft_lds_2d(T2 *a, T2 *b, int S, int ss, int es, const FftSched &sc, const T2 *__restrict__ tw,
                          int tid, int nt) {
    const int L = sc.L;
    const uint32_t mS = S <= 1 ? 0u : 0xFFFFFFFFu / (uint32_t)S + 1u;   // ceil(2^32 / S)
    for (int p = 0; p < sc.np; ++p) {
        const FftPass &ps = sc.ps[p];
        switch (ps.R) {
            case 2: stockham_pass_2d<T, T2, 2, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
            case 3: stockham_pass_2d<T, T2, 3, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
            case 4: stockham_pass_2d<T, T2, 4, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
            case 5: stockham_pass_2d<T, T2, 5, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
            case 8: stockham_pass_2d<T, T2, 8, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
            default:
                if constexpr (RMAX >= 16) {
                    switch (ps.R) {
                        case 6: stockham_pass_2d<T, T2, 6, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
                        case 9: stockham_pass_2d<T, T2, 9, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
                        case 10: stockham_pass_2d<T, T2, 10, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
                        case 12: stockham_pass_2d<T, T2, 12, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
                        case 15: stockham_pass_2d<T, T2, 15, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
                        default: stockham_pass_2d<T, T2, 16, DIR>(a, b, S, mS, L, ss, es, ps, tw, tid, nt); break;
                    }
                }
                break;
        }
        __syncthreads();
        T2 *t = a;
        a = b;
        b = t;
    }
    return a;
}

// Copy a length-L twiddle table into LDS (caller synchronises before use).
template <typename T2>
__device__ __forceinline__ void stage_twiddles(T2 *dst, const T2 *__restrict__ src, int L, int tid, int nt) {
    for (int i = tid; i < L; i += nt) dst[i] = src[i];
}

// blockIdx -> logical tile so that the blocks resident on one XCD (hardware hands
// block i to XCD i mod 8) work on one contiguous range of tiles and share L2 lines.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
    const int nx = 8;
    const int q = nblocks / nx, r = nblocks % nx;
    const int x = bid % nx, local = bid / nx;
    return x * q + (x < r ? x : r) + local;
}

// Plan groups: one grid over the workgroups of several plans, start[] their offsets
// (start[n] = the total); the member owning workgroup g is the largest i with start[i] <= g.
__device__ __forceinline__ int group_member(const int *__restrict__ start, int n, int g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Block-wide sum of up to 4 FP64 values per thread in a fixed order (deterministic):
// wave64 butterfly shuffles, then the waves' results added in wave order by thread 0.
// red: LDS scratch of >= 16 K doubles (up to 16 waves).  Result valid in thread 0.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *red, int tid, int nt) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        v[k] = x;
    }
    const int w = tid >> 6, nw = (nt + 63) >> 6;
    if ((tid & 63) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[k * 16 + w] = v[k];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int i = 0; i < nw; ++i) s += red[k * 16 + i];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Sum of n partials (fixed order) by a whole block; result broadcast to all threads.
__device__ __forceinline__ double block_sum_partials(const double *__restrict__ p, int n,
                                                     double *red, int tid, int nt) {
    double v[1] = {0.0};
    // four strided loads in flight per step; each thread adds its partials in index order
    for (int i0 = tid; i0 < n; i0 += 4 * nt) {
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = i0 + u * nt < n ? p[i0 + u * nt] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * nt < n) v[0] += x[u];
    }
    block_sum<1>(v, red, tid, nt);
    if (tid == 0) red[64] = v[0];
    __syncthreads();
    double s = red[64];
    __syncthreads();
    return s;
}

// Sums of K <= 5 arrays of n partials each by a whole block, all in one pass and one
// tree (the same per-array order as block_sum_partials); results broadcast to all
// threads.  red: >= 96 doubles.
// Array k holds n[k] partials (the arrays of one chain may come from passes with
// different tile counts); with equal counts the order is that of a single count.
template <int K>
__device__ __forceinline__ void block_sum_partials_k(const double *const (&p)[K], const int (&n)[K], double (&out)[K],
                                                     double *red, int tid, int nt) {
    static_assert(K >= 1 && K <= 5, "block_sum uses red[k * 16 + wave] and red[80 + k]");
    double v[K];
    int nmax = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = 0.0;
        nmax = n[k] > nmax ? n[k] : nmax;
    }
    // four strided loads per array in flight per step; each thread adds its partials of
    // every array in index order (the order of one load at a time)
    for (int i0 = tid; i0 < nmax; i0 += 4 * nt) {
        double x[4][K];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) x[u][k] = i0 + u * nt < n[k] ? p[k][i0 + u * nt] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (i0 + u * nt < n[k]) v[k] += x[u][k];
    }
    block_sum<K>(v, red, tid, nt);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[80 + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = red[80 + k];
    __syncthreads();
}

}  // namespace msb
