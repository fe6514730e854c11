// The fused solver epilogue of the product kernels (shared by the x-inverse pass of
// the chain and the tiled single-pass product).
#pragma once

#include "passes.hpp"

namespace msb {

// Store of a kernel result through the L2 to the memory side: a relaxed agent-scope store,
// which the compiler emits as a vector store with the sc1 (write-through) bit.  The block
// kernels' plain product writes its output this way when the whole output fits well within
// the L2s: the results then reach memory while the blocks run rather than in the L2
// write-back that ends the kernel (0.45 of 8.5 us on the one-case 512^2 FP64 product).  Not
// for outputs that the next kernel reads back (the fused CG and Verlet vectors, whose reads
// hit the L2 lines a plain store leaves behind: write-through made those steps 20-35% slower)
// or that exceed the L2s (16 cases of 512^2: 3% slower).
template <typename T> __device__ __forceinline__ void st_wt(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The fused epilogue at one DOF: f = (A u) at addr (corrections applied), fx = the DOF
// is constrained; pa_idx indexes the per-case array e.pa (the ADR density).
template <typename T>
__device__ __forceinline__ void epilogue_at(const EndArgs<T> &e, const T *__restrict__ uin, size_t addr, size_t pa_idx,
                                            T f, bool fx, T sign, T rinv, T dth, double &acc0, double &acc1,
                                            double &acc2) {
    switch (e.epi) {
        case EPI_APPLY:
            if (e.wt)
                st_wt(&e.out[addr], fx ? T(0) : sign * f);
            else
                e.out[addr] = fx ? T(0) : sign * f;
            break;
        case EPI_CG_Q: {
            const T q = fx ? T(0) : -f;
            e.out[addr] = q;
            const double qd = (double)q;
            acc0 += (double)uin[addr] * qd;
            acc1 += (double)e.rhs[addr] * qd;
            acc2 += qd * qd;
            break;
        }
        case EPI_PCG_Z: {
            const T z = fx ? T(0) : sign * f;
            e.out[addr] = z;
            acc0 += (double)uin[addr] * (double)z;
            break;
        }
        case EPI_ADR: {
            // F = f + b; K1 = -(F - F_prev) / (D v) where v != 0 (the local
            // stiffness of the adaptive damping); sums u.K1.u and u.u
            if (fx) {
                e.out[addr] = T(0);
                break;
            }
            const T Fn = f + e.rhs[addr];
            if (e.part) {   // no partials on the first evaluation (no previous F)
                const double uu = (double)uin[addr];
                const double vv = (double)e.ev[addr];
                if (vv != 0.0) {
                    const double Dd = (double)e.pa[pa_idx];
                    acc0 += uu * uu * (-((double)Fn - (double)e.out[addr]) / (Dd * vv));
                }
                acc1 += uu * uu;
            }
            e.out[addr] = Fn;
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
            if (e.u_next) {   // Alg. 2's displacement update of the next step (the prologue's arithmetic)
                const T dtt = T(e.dt), hdt2 = T(0.5 * e.dt * e.dt);
                e.u_next[addr] = fx ? (e.pg ? e.pg[addr] : T(0)) : uin[addr] + dtt * vn + hdt2 * an;
            }
            break;
        }
        default:  // EPI_DOT
            if (!fx) acc0 += (double)e.rhs[addr] * (double)f;
            break;
    }
}


}  // namespace msb
