// Kernel arguments and launchers of the FFT product passes (A u = A_hat u + D^e u +
// D^f u, masked on constrained DOFs).  Implemented in passes.hip.
#pragma once

#include "common.hpp"

namespace msb {

// Largest workgroup of the product kernels (their launch bound): 512 threads leave the
// compiler 256 VGPRs per lane, which the FP64 radix-16 passes need without spilling.
constexpr int kMaxBlock = 512;

// What the x-forward pass does to its input rows before transforming them.
enum Prologue : int {
    PRO_NONE = 0,   // transform u as given
    PRO_CG_P = 1,   // fused CG step: x += alpha p, r -= alpha q, p <- r + beta p, transform p
    PRO_VV_U = 2,   // u <- u + dt v + dt^2 a / 2, u_C <- g_C, store u, transform u
    PRO_PCG_R = 3,  // preconditioned CG, preconditioner chain: x += alpha p, r -= alpha q, transform r
    PRO_PCG_P = 4,  // preconditioned CG, stiffness chain: p <- z + beta p, transform p
    PRO_ADR_U = 5,  // dynamic relaxation (Alg. 1): v <- ((2 - c) v + 2 F/D)/(2 + c), u <- u + v, transform u
};

// What the x-inverse pass does with f = A u after the corrections.
enum Epilogue : int {
    EPI_APPLY = 0,  // out = sign * f, 0 on constrained DOFs
    EPI_CG_Q = 1,   // out = q = -f (K p), 0 on constrained; partials p.q, r.q, q.q
    EPI_RESID = 2,  // out = rhs + f, 0 on constrained; partial out.out
    EPI_VV = 3,     // a' = (f + b)/rho; v += dt (a + a')/2; a = a'; energy partials
    EPI_DOT = 4,    // no output; partial w.f over free DOFs
    EPI_PCG_Z = 5,  // out = z = sign * f (the preconditioned residual), 0 on constrained; partial r.z
    EPI_ADR = 6,    // out = F = f + b (0 on constrained); partials u.K1.u, u.u of the adaptive damping
};

template <typename T> struct PassArgs {
    // geometry
    int d, B, Nx, Ny, Nz, M;
    int rows;            // Ny*Nz per case
    int H;               // Lx/2 + 1
    int Ly, Lz;
    int F;               // rows per workgroup (x passes)
    int Fl;              // lines per workgroup (line passes)
    int wave_x, wave_l;  // 1: wave-owned signals, 0: whole-block teams (x passes / line passes)
    int spw, spw_i, lpw; // wave mode: complex slots per wave (x-forward, x-inverse), lines per wave (line passes)
    int ip_x, ip_l;      // 1: in-place Stockham stages (one LDS signal buffer) in the x / line passes
    int bthreads;        // block mode: threads per block (x and y passes)
    int bthreads_line;   // block mode: threads per block of the 2D line pass
    int N;               // nodes per case
    int corr;            // 1: add the corrections D^e and D^f (0 for the preconditioner's spectral operator)
    FftSched sx, sy, sz;
    const cplx_t<T> *twx, *twy, *twz;
    cplx_t<T> *T1, *T2;
    // operator
    const T *spec;       // [slots][ncomp][H][Ly][Lz]
    size_t spec_slot;    // stride between slots (0 = shared by all cases)
    const T *de;         // [slots][ncomp][(M+1)^(2d)]
    size_t de_slot;
    const T *w;          // [slots][ncomp][n_off]
    size_t w_slot;
    int de_stride;       // (M+1)^(2d)
    int n_off;
    // surface correction: per-node factors [N] (null: off) and the stencil offsets
    // [n_off][3] in the order of the weight table w
    const T *nu;
    const int32_t *offs;
    // constraints and bonds
    const uint8_t *fixed;          // [d][N] or null
    const uint8_t *row_fix;        // [d][rows] with fixed: per x-row 0 none constrained, 1 all, 2 some
    const int32_t *fix_sat;        // 2D with fixed: [(Ny + 1)][(Nx + 1)] summed-area table of the mask
    const int32_t *br_row_ptr;     // [rows+1] or null
    const int32_t *br_node_i;
    const int32_t *br_bond_ptr;
    const int32_t *br_q;
    const int32_t *br_off;
    // Tiled single-pass product (2D): frame length tl per axis (0: the global chain of
    // passes), tiles per case along x and y, threads per workgroup, the frame's Stockham
    // schedule and twiddles, and the frame spectra [slots][3][tl][tl] ((Gxx+Gyy)/2,
    // (Gxx-Gyy)/2, Gxy of the generating array wrapped to tl x tl, scaled by 1/tl^2)
    int tl, ttx, tty, tthreads;
    int treg;            // 1: the register-resident frame kernel (tl = 16, 32 or 64)
    int tper;            // register kernel: consecutive tiles per workgroup (loads of the next overlap the current)
    FftSched stl;
    const cplx_t<T> *twt;
    const T *tspec;
    const T *tspecr;     // the same spectra in the register-frame thread order (tl = 16, 32, 64)
    size_t tspec_slot;
    // slots per case of the epilogue partial sums: the x-inverse tiles of the chain, or
    // the tiles of the tiled product
    int ept;
};

// Per-call data of the prologue/epilogue.
template <typename T> struct EndArgs {
    int pro, epi;
    // prologue
    T *pio;              // PRO_CG_P, PRO_PCG_P: p (in/out); PRO_VV_U, PRO_ADR_U: u (in/out)
    const T *pr;         // PRO_CG_P: r;          PRO_VV_U: v;  PRO_PCG_R: p;  PRO_PCG_P: z
    const T *pa;         // PRO_VV_U: a;  PRO_ADR_U, EPI_ADR: the fictitious density D
    size_t pa_stride;    // PRO_ADR_U, EPI_ADR: stride of D between cases (0: shared)
    const T *pg;         // PRO_VV_U: g or null
    // PRO_CG_P (single-reduction CG): alpha = r.r / p.q, r'.r' = r.r - 2 alpha r.q +
    // alpha^2 q.q, beta = r'.r' / r.r from the partial sums of the previous iteration
    T *cx;                     // x (updated); PRO_ADR_U: the velocity (updated)
    T *cr;                     // r (updated)
    const T *cq;               // q = K p of the previous iteration; PRO_ADR_U: F of the current u
    const double *cg3;         // previous x-inverse partials [3][B*tiles]: p.q, r.q, q.q
    const double *rr_prev;     // previous true r.r partials [B][tiles]
    double *rr_out;            // this iteration's true r.r partials [B][tiles]
    const double *case4;       // if set: [B][K] case sums already reduced (K and order as the
                               // prologue reduces them: CG_P r.r p.q r.q q.q; PCG_R r.r r.z p.q
                               // r.q q.q; PCG_P r.z r.z_prev)
    // PRO_PCG_R / PRO_PCG_P: r.z partials [B][tiles] of this and the previous iteration
    const double *rz_k, *rz_km1;
    const double *beta_num;    // first iteration of a continued run: beta = sum(num)/sum(den)
    const double *beta_den;
    int n_num, n_den;
    int first;                 // no pending update (first iteration)
    int update_only;           // apply the pending update and stop (no transform)
    int no_transform;          // apply the prologue (update, store, partials, flags) only: the
                               // tiled product transforms the stored vector afterwards
    // slots per case (n_cg3) and stride between the arrays (s_cg3) of the epilogue partials
    // cg3 the prologue reduces (they come from the previous product's epilogue, whose
    // tiles may differ from the x tiles of this launch); 0: this launch's x tiles
    int n_cg3;
    size_t s_cg3;
    // fused CG step in the frame-16 register kernel (cg_fused): the update of the previous
    // step is applied on the patch as it loads, from the previous vectors pio (p), cr (r),
    // cq (q) and the case sums case4; the new p and r of the block's inner nodes go to
    // p_new / r_new (patches overlap: the previous vectors stay readable), x is updated in
    // place, q = K p to out; r.r of the block's inner nodes to rr_out[block].  rr_tiles:
    // the unfused CG epilogue also writes the r.r of the block's inner nodes (r = rhs) to
    // rr_out[block], so that a fused step can follow.
    // cg_fused = 2: the stiffness step of preconditioned CG, p = z + beta p (z in pr, the
    // previous p in pio, beta = r.z / previous r.z from case4), p of the inner nodes to p_new,
    // then q = K p (in place: no block reads q off its own nodes) and its partials
    T *p_new;
    T *r_new;
    int cg_fused;
    int rr_tiles;
    int *iters;                // [B] completed updates
    const int *case_done;      // [B] per-case stop flags (skip work) or null
    // CG chains keep the flags in two arrays by iteration parity: the x-forward stops on
    // done_prev (the flags before this iteration) and writes every case's new flag into
    // done_rw, which the later passes read as case_done.  A block that starts after
    // another block of its case has flagged convergence in the same launch therefore
    // still applies its share of the final update.
    const int *done_prev;      // flags before this iteration, or null (stop on case_done)
    int *done_rw;              // PRO_CG_P, PRO_PCG_R: the new flags
    const double *thresh;      // PRO_CG_P: per-case stop threshold on r.r (or null)
    double dt;
    // epilogue
    const T *uin;        // the vector that was transformed (for D^e, D^f, dots)
    T *out;              // EPI_APPLY/CG_Q/RESID output
    const T *rhs;        // EPI_RESID rhs; EPI_VV b; EPI_DOT w; EPI_CG_Q r
    T *ev;               // EPI_VV: v
    T *ea;               // EPI_VV: a
    T *u_next;           // EPI_VV: if set, the next step's displacement u + dt v' + dt^2/2 a' (g on
                         // constrained DOFs, pg) into this vector, so that the next product needs
                         // no prologue pass (u itself is read by neighbouring blocks: not in place)
    double sign;         // EPI_APPLY sign
    int wt;              // EPI_APPLY in the block kernels: the output written through the L2 (set
                         // by the block-kernel launcher, see st_wt)
    double rho;
    int energy;          // EPI_VV: accumulate energy partials
    double *part;        // partial sums [K][B*tiles]
};

// Launch the pass chain on stream s.  ev (optional, npasses+1 events) is recorded
// before the first kernel and after each kernel (measurement only); with reps > 1 each
// kernel is launched reps times back to back between its events (measurement only: the
// outputs of repeated in-place passes are not the product).
template <typename T>
msb_status launch_product(const PassArgs<T> &a, const EndArgs<T> &e, hipStream_t s,
                          hipEvent_t *ev = nullptr, int reps = 1);
// The tiled single-pass 2D product kernel over B x ttx x tty tiles (tile.hip): lds
// dynamic bytes per workgroup, composite: the frame schedule uses a composite radix;
// launched reps times back to back (reps > 1: measurement only).
template <typename T>
hipError_t launch_tile_kernel(const PassArgs<T> &a, const EndArgs<T> &e, size_t lds, bool composite, int reps,
                              hipStream_t st);
inline int n_passes(int dim) { return dim == 2 ? 3 : 5; }
// Kernels a product launch times: the chain's passes, or the one tiled kernel.
template <typename T> inline int n_passes(const PassArgs<T> &a) { return a.tl > 0 ? 1 : n_passes(a.d); }
// Tiles per case of the tiled product for frame length tl (0 when tl is 0).
int tile_count(const msb_plan_s *p, int tl);
// Slots per case every epilogue partial array needs under any valid configuration.
int64_t partial_slots(const msb_plan_s *p);

// Arguments of the product passes for plan p and operator op, with the plan's launch
// configuration for T's precision, or cfg (and its radix cap) when given.
template <typename T>
PassArgs<T> pass_args(const msb_plan_s *p, const DeviceOp &op, const msb_launch_config *cfg = nullptr);

// Group launch: one grid per pass over the tiles of n plans that share the dimension
// and the launch configuration.  start_*: device [n + 1] tile offsets of each pass
// (start[n] = total); lds_*: the largest member's dynamic LDS per pass.
struct GroupGrid {
    int n = 0;
    const int *start_x = nullptr, *start_l = nullptr, *start_y = nullptr;
    int total_x = 0, total_l = 0, total_y = 0;
    size_t lds_x = 0, lds_l = 0, lds_y = 0;
    // tiled group products (2D, tile > 0): one launch of the tiled kernel over the members'
    // blocks (table start_t), preceded by the transform-free x pass when pro is set (the
    // end arguments carry a solver prologue)
    const int *start_t = nullptr;
    int total_t = 0;
    size_t lds_t = 0;
    int tiled = 0, pro = 0;
    int cgq = 0;   // CG slots: the tiled kernel's CG-epilogue form (with or without a prologue)
};
// a: any member's host arguments (for the common geometry); dA/dE: device arrays of the
// members' arguments; composite: some member's schedules use a composite radix.
template <typename T>
msb_status launch_group(const PassArgs<T> &a, const GroupGrid &gg, const PassArgs<T> *dA, const EndArgs<T> *dE,
                        bool composite, hipStream_t st);
// Per-case tile counts of a plan's passes under a configuration: x passes, line
// product (2D y / 3D z), 3D y passes, blocks of the tiled product (2D, tile > 0, else 0);
// and their dynamic LDS bytes.
void pass_tiles(const msb_plan_s *p, const msb_launch_config &c, bool fp32, int tiles[4], size_t lds[4]);
// The tiled kernel over the blocks of a group's members (tile.hip): a, any member's host
// arguments (frame length and kernel form, shared by the members).
template <typename T>
hipError_t launch_tile_group(const PassArgs<T> &a, const GroupGrid &gg, const PassArgs<T> *dA, const EndArgs<T> *dE,
                             bool composite, hipStream_t st);
// Whether a plan's schedules at radix cap max_radix use a composite radix.
bool plan_needs_composite(const msb_plan_s *p, bool fp32, int max_radix);

// tiles of the x passes per case (partial-sum slots per case)
int x_tiles_per_case(const msb_plan_s *p, int F);

}  // namespace msb
