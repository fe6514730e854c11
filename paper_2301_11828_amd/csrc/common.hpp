// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/msbfm.h"

namespace msb {

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...);

#define MSB_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::msb::set_error("%s:%d %s failed: %s", __FILE__, __LINE__, #call,          \
                             hipGetErrorString(e_));                                    \
            return MSB_EDEVICE;                                                         \
        }                                                                               \
    } while (0)

#define MSB_CHECK(cond, status, ...)                                                    \
    do {                                                                                \
        if (!(cond)) {                                                                  \
            ::msb::set_error(__VA_ARGS__);                                              \
            return (status);                                                            \
        }                                                                               \
    } while (0)

#define MSB_TRY(expr)                                                                   \
    do {                                                                                \
        msb_status s_ = (expr);                                                         \
        if (s_ != MSB_OK) return s_;                                                    \
    } while (0)

// ------------------------------------------------------------------ complex types
template <typename T> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };
template <typename T> using cplx_t = typename cplx_of<T>::type;

// ------------------------------------------------------------------ FFT schedule
constexpr int kMaxPasses = 12;

// One transform axis: length L = product of radix[0..np); the radices are among
// {2,3,4,5,8} and, with a radix cap of 16, {6,9,10,12,15,16}.
// Twiddle table tw[t] = exp(-2 pi i t / L), t < L (device, both precisions).
struct FftAxis {
    int L = 0;
    int np = 0;                       // FP64 schedule
    int radix[kMaxPasses] = {};
    int np32 = 0;                     // FP32 schedule (may use the composite radices)
    int radix32[kMaxPasses] = {};
    double2 *tw64 = nullptr;
    float2 *tw32 = nullptr;
};

// Division by a runtime constant d < 2^16 for numerators < 2^16:
// q = umulhi(n, ceil(2^32/d)) is exact in that range (m = 0 encodes d = 1).
inline uint32_t div_magic(uint32_t d) { return d <= 1 ? 0u : (uint32_t)((((uint64_t)1 << 32) + d - 1) / d); }

// Per-pass constants of a Stockham schedule (kernel argument, by value).
struct FftPass {
    int R;          // radix
    int Ns;         // points already combined (product of earlier radices)
    int nb;         // butterflies per signal, L / R
    int twstep;     // L / (Ns R)
    uint32_t m_nb;  // div_magic(nb)
    uint32_t m_Ns;  // div_magic(Ns)
};

struct FftSched {
    int L;
    int np;
    FftPass ps[kMaxPasses];
};

inline FftSched sched_of(const FftAxis &a, bool fp32 = false) {
    FftSched s{};   // unused passes zero: argument blocks compare bytewise (cached solver graphs)
    s.L = a.L;
    s.np = fp32 ? a.np32 : a.np;
    const int *radix = fp32 ? a.radix32 : a.radix;
    int Ns = 1;
    for (int i = 0; i < kMaxPasses; ++i) {
        FftPass &p = s.ps[i];
        if (i < s.np) {
            p.R = radix[i];
            p.Ns = Ns;
            p.nb = a.L / p.R;
            p.twstep = a.L / (Ns * p.R);
            p.m_nb = div_magic((uint32_t)p.nb);
            p.m_Ns = div_magic((uint32_t)Ns);
            Ns *= p.R;
        } else {
            p = FftPass{1, 1, 1, 1, 0u, 0u};
        }
    }
    return s;
}

template <typename T> inline const cplx_t<T> *tw_of(const FftAxis &a);
template <> inline const double2 *tw_of<double>(const FftAxis &a) { return a.tw64; }
template <> inline const float2 *tw_of<float>(const FftAxis &a) { return a.tw32; }

// Factor L into the fewest stages with radix <= rmax from the supported set;
// returns false if L has a prime factor other than 2, 3, 5.
bool factor_length(int L, std::vector<int> &radices, int rmax);
// Smallest L >= nmin whose prime factors are all in {2,3,5} (and even when even_only).
int next_smooth(int nmin, bool even_only);

// ------------------------------------------------------------------ operators
// Device data of the operator A for one or more sets of influence coefficients,
// stored as `count` back-to-back slots (slot = batch case when every case has its
// own coefficients, else a single shared slot).
// Spectra of the generating array wrapped to a tl x tl frame (tiled 2D product), one
// set per frame length in use: [count][3][tl][tl] = (Gxx+Gyy)/2, (Gxx-Gyy)/2, Gxy,
// scaled by 1/tl^2.
struct TileSpec {
    int tl = 0;
    double *s64 = nullptr;   // [slots][3][tl][tl]
    float *s32 = nullptr;
    // frames with register-resident transforms (tl = R S: 16, 32, 64): the same values in the
    // order the kernel's threads load them, [slots][3][R][S tl], entry (i, t) = spectrum at
    // ky = t mod tl, kx = t div tl + S i (each register's loads are one contiguous run)
    double *r64 = nullptr;
    float *r32 = nullptr;
};

struct DeviceOp {
    int count = 0;
    double *spec64 = nullptr;   // [count][ncomp][H][Ly][Lz] real spectra, scaled by 1/prod(L)
    float *spec32 = nullptr;
    double *de64 = nullptr;     // [count][ncomp][(M+1)^(2d)] incomplete-horizon diagonal table
    float *de32 = nullptr;
    double *w64 = nullptr;      // [count][ncomp][n_off] bond weights (broken-bond correction)
    float *w32 = nullptr;
    std::vector<TileSpec> tiles;   // frame spectra for the tiled product (2D), built on demand
    std::vector<std::vector<double>> infl_slots;   // the coefficients of every slot (tile spectra rebuilds)
};

}  // namespace msb

struct msb_plan_s {
    // problem
    int dim = 2;
    int64_t n[3] = {1, 1, 1};
    int64_t N = 0;              // nodes per case
    double h = 1.0;
    int M = 1;
    double alpha = 0.0;
    std::vector<double> infl;   // shared coefficients (n_infl), empty = omega 1
    std::vector<double> infl_case;  // [B][n_infl] when per-case
    int n_infl = 0;
    bool per_case = false;
    double rho = 1.0;
    int B = 1;
    int ncomp = 3;              // d(d+1)/2 block components: 2D xx,xy,yy; 3D xx,xy,xz,yy,yz,zz
    int device = 0;

    // FFT
    int64_t L[3] = {1, 1, 1};
    int64_t H = 1;              // L[0]/2 + 1 (half spectrum along x)
    msb::FftAxis ax[3];
    std::vector<msb::FftAxis> tax;   // frame axes (twiddles) of the tiled product, per length in use
    msb_launch_config cfg[2];   // launch configuration of the product: [0] FP64, [1] FP32

    // stencil (host)
    int n_off = 0;
    std::vector<int> off;       // [n_off][3]
    int de_stride = 0;          // (M+1)^(2d)

    // operators: op = A for the current coefficients (one slot, or B slots when
    // per_case); dop[k] = derivative operator for omega = (r/delta)^k (built lazily)
    msb::DeviceOp op;
    std::vector<msb::DeviceOp> dop;
    msb::DeviceOp pre;          // circulant preconditioner spectra (built on first use)

    // surface correction (Remark 3, eq. (scr)): per-node factors nu, device [N] in both
    // precisions, or null; stencil offsets on the device for the correction pass
    double *nu64 = nullptr;
    float *nu32 = nullptr;
    std::vector<double> nu_host;     // [N] or empty
    int32_t *off_dev = nullptr;      // [n_off][3]

    // constraints
    uint8_t *fixed = nullptr;   // device [d][N] or null
    uint8_t *row_fix = nullptr; // device [d][Ny Nz]: per x-row, 0 no constrained DOF, 1 all, 2 some
    int32_t *fix_sat = nullptr; // 2D: device [(Ny + 1)][(Nx + 1)] constrained DOFs in [0, x) x [0, y)
    int64_t n_fixed = 0;

    // broken bonds (device), grouped by grid row (row = k*Ny + j)
    int64_t n_pairs = 0;
    int32_t *br_row_ptr = nullptr;   // [rows+1] -> range in br_node
    int32_t *br_node_i = nullptr;    // [nbr] node id (within a case), sorted
    int32_t *br_bond_ptr = nullptr;  // [nbr+1] -> range in br_q / br_off
    int32_t *br_q = nullptr;         // [ndir] neighbour node id
    int32_t *br_off = nullptr;       // [ndir] stencil offset id
    int64_t n_br_nodes = 0;
    std::vector<int64_t> bonds_host; // [n_pairs][2] the broken set, p < q, sorted

    // crack propagation (crack.hip): broken-bond bit mask over the half stencil
    // (offsets o with p + o > p), one bit per bond {p, p + o}; rebuilt from bonds_host
    // when stale
    uint32_t *mu_mask = nullptr;     // [N][mu_words]
    int mu_words = 0;
    bool mu_valid = false;
    void *crack_ws = nullptr;        // crack.hip workspace

    // workspace (device)
    void *T1 = nullptr;         // complex [B][d][Nz][H][Ny] (largest precision)
    void *T2 = nullptr;         // 3D only: complex [B][d][H][Ly][Nz]
    size_t T1_bytes = 0, T2_bytes = 0;

    // solver vectors, partial sums and pinned mirrors (solver translation unit)
    void *solver_cache = nullptr;
    // incremented whenever A changes (coefficients, bonds, surface factors, constraints)
    int64_t op_version = 0;
    // incremented whenever the padded lengths (and with them the transform layout) change
    int64_t layout_version = 0;
};

namespace msb {

int64_t rows_total(const msb_plan_s *p);   // Ny * Nz grid rows per case
size_t spectrum_len(const msb_plan_s *p);  // H * Ly * Lz reals per component
size_t de_len(const msb_plan_s *p);        // ncomp * (M+1)^(2d) per slot
size_t w_len(const msb_plan_s *p);         // ncomp * n_off per slot

// Launch configurations (passes.hip): the size-based default, and the check that
// a configuration fits the hardware limits and the schedules' index arithmetic.
msb_launch_config default_config(const msb_plan_s *p, bool fp32);
msb_status check_config(const msb_plan_s *p, bool fp32, const msb_launch_config &c);
// Stockham schedules of every axis for one precision with radices <= max_radix (plan.cpp).
msb_status set_schedules(msb_plan_s *p, bool fp32, int max_radix);
// The schedule of one axis for a given radix cap, leaving the plan's own unchanged.
FftSched make_sched(const FftAxis &ax, bool fp32, int max_radix);
// New padded lengths: rebuild twiddles, spectra and transform workspace (plan.cpp).
msb_status relayout(msb_plan_s *p, const int64_t *L);

msb_status alloc_operator(msb_plan_s *p, DeviceOp &op, int count);
msb_status build_preconditioner(msb_plan_s *p);   // (re)builds p->pre
msb_status build_preconditioners(msb_plan_s *const *ps, int n);   // parallel host work, plans without one
msb_status set_infl_many(msb_plan_s *const *ps, int n, const double *const *infl, int n_infl, const int *per_case);
// Fictitious density of dynamic relaxation, D_ii = 1/4 sum_j |K_ij| for every DOF of
// every operator slot ([slots][d][N]; slots = per-case operators or 1) (plan.cpp).
void build_adr_density(const msb_plan_s *p, std::vector<double> &D, int &slots);
msb_status fill_operator(msb_plan_s *p, const std::vector<double> &infl, DeviceOp &op, int slot);
void free_operator(DeviceOp &op);
// Frame spectra of every operator of the plan (op and the derivative operators) and the
// frame axis for the tile lengths of both launch configurations and `extra` (if > 0);
// host work and uploads, so never during graph capture (plan.cpp).
// Frame spectra for the plan's configured tile lengths and `extra` (all operators; for
// `extra` only the stiffness operator when extra_op_only: a plan group's frame length).
msb_status ensure_tiles(msb_plan_s *p, int extra = 0, bool extra_op_only = false);
const TileSpec *find_tile_spec(const DeviceOp &op, int tl);
const FftAxis *find_tile_axis(const msb_plan_s *p, int tl);
void solver_cache_free(msb_plan_s *p);
// Replace the broken set by pairs[nb][2] (validated), rebuild the D^f lists (plan.cpp).
msb_status set_bonds_impl(msb_plan_s *p, const int64_t *pairs, int64_t nb);
void crack_free(msb_plan_s *p);   // crack.hip

}  // namespace msb
