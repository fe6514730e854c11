/*
 * CPU oracle for the linear bond-based peridynamic force, FP64, plain C.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * GPU library.
 *
 * What it computes is the plain meshfree sum of Sec. 2.3, eq. (mat:f1):
 *
 *     f_p = sum_{q in B_delta(x_p) cap Omega, q != p}
 *              mu_pq * C(x_q - x_p) * (u_q - u_p) * lambda_q * V_q
 *
 * with the micromodulus tensor of eq. (ker:e1), C(xi) = alpha xi (x) xi / |xi|^3,
 * optionally scaled by a radial influence function omega(|xi|/delta) =
 * sum_k a_k (|xi|/delta)^k (omega == 1 when no coefficients are given, which is
 * the paper's case), the partial-volume factor lambda of eq. (fac:e1), the
 * uniform node volume V = h^d (Sec. 3, Sec. 4) and the bond status mu of
 * eq. (mu) (0 for a bond in the broken list, 1 otherwise).
 *
 * Readings taken where the paper leaves room:
 *   - nodes sit at x_i = (i + 1/2) h, 0-based (Sec. 3 uses 1-based (i - 1/2) h);
 *   - horizon membership |xi| <= delta is decided on the integer offset,
 *     |o|^2 <= M^2 with delta = M h, so there are no floating-point ties;
 *   - lambda uses the form of eq. (fac:e1) (grid spacing Delta x = h); the
 *     index-unit form printed in eq. (tra:e2) is not continuous and is not used;
 *     its first branch |xi| <= delta - h/2 is, on integer offsets,
 *     |o|^2 <= M^2 - M.
 *
 * The loop visits, for each node p, the offsets with |o_i| <= M per axis: the
 * block-banded-block bound of eq. (band).  Nothing is precomputed per offset;
 * every bond weight is evaluated from the node coordinates.
 *
 * Surface correction (Remark 3, eq. (scr)), when per-node factors nu are given:
 * on the rows of Omega_e (nodes whose horizon leaves the grid: within M of a
 * face) every bond is scaled by v_pq = (nu_p + nu_q) / 2; other rows unchanged.
 * The paper leaves v_pq to the cited surface-correction method; the average of
 * per-node factors is the reading taken here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* is q in the sorted broken-neighbour list of p? (bond status mu = 0) */
static int bond_broken(int64_t p, int64_t q, const int64_t *br_ptr, const int64_t *br_idx)
{
    if (!br_ptr) return 0;
    int64_t lo = br_ptr[p], hi = br_ptr[p + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (br_idx[mid] == q) return 1;
        if (br_idx[mid] < q) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/*
 * d x d bond tensor W = mu * alpha * omega * lambda * V * xi xi^T / |xi|^3 for the
 * ordered pair (p, q) given by node indices.  Returns 0 when q is outside the
 * horizon of p (or q == p), 1 otherwise (W filled, possibly zero if broken).
 */
static int bond_tensor(int dim, const int64_t ip[3], const int64_t iq[3], double h, int M,
                       double alpha, int n_infl, const double *infl, double W[3][3])
{
    int64_t s2 = 0;
    for (int a = 0; a < dim; ++a) {
        int64_t o = iq[a] - ip[a];
        s2 += o * o;
    }
    if (s2 == 0 || s2 > (int64_t)M * M) return 0;

    double delta = M * h;
    double xi[3] = {0, 0, 0}, r2 = 0.0;
    for (int a = 0; a < dim; ++a) {
        double xp = (ip[a] + 0.5) * h;
        double xq = (iq[a] + 0.5) * h;
        xi[a] = xq - xp;
        r2 += xi[a] * xi[a];
    }
    double r = sqrt(r2);

    /* eq. (fac:e1): full volume inside delta - h/2, linear ramp to delta */
    double lam;
    if (s2 <= (int64_t)M * M - M) lam = 1.0;
    else lam = (2.0 * delta + h - 2.0 * r) / (2.0 * h);

    /* radial influence, omega(r/delta) = sum_k a_k (r/delta)^k */
    double om = 1.0;
    if (n_infl > 0) {
        om = 0.0;
        for (int k = 0; k < n_infl; ++k) om += infl[k] * pow(r / delta, (double)k);
    }

    double V = 1.0;
    for (int a = 0; a < dim; ++a) V *= h;

    double c = alpha * om * lam * V / (r2 * r);
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) W[a][b] = c * (xi[a] * xi[b]);
    return 1;
}

static void node_index(int64_t p, const int64_t n[3], int64_t ip[3])
{
    ip[0] = p % n[0];
    ip[1] = (p / n[0]) % n[1];
    ip[2] = p / (n[0] * n[1]);
}

/*
 * Force at a list of nodes (or at every node when rows == NULL), eq. (mat:f1).
 *   u    : [dim][N] displacement, SoA, node id = (k*ny + j)*nx + i
 *   f    : [dim][nrows] output (nrows = N when rows == NULL)
 *   br_ptr/br_idx : per-node sorted list of broken neighbours (CSR), or NULL
 */
void oracle_force_rows(int dim, const int64_t *n, double h, int M, double alpha,
                       int n_infl, const double *infl, const double *u,
                       const int64_t *br_ptr, const int64_t *br_idx,
                       const int64_t *rows, int64_t nrows, const double *nu, double *f)
{
    int64_t nn[3] = {n[0], n[1], dim == 3 ? n[2] : 1};
    int64_t N = nn[0] * nn[1] * nn[2];
    if (!rows) nrows = N;
    int64_t Mz = dim == 3 ? M : 0;

#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t p = rows ? rows[r] : r;
        int64_t ip[3], iq[3];
        node_index(p, nn, ip);
        double acc[3] = {0, 0, 0};
        int on_e = 0;   /* p in Omega_e: within M of a face of the grid */
        for (int a = 0; a < dim; ++a)
            if (ip[a] < M || ip[a] >= nn[a] - M) on_e = 1;
        for (int64_t oz = -Mz; oz <= Mz; ++oz)
            for (int64_t oy = -M; oy <= M; ++oy)
                for (int64_t ox = -M; ox <= M; ++ox) {
                    iq[0] = ip[0] + ox; iq[1] = ip[1] + oy; iq[2] = ip[2] + oz;
                    if (iq[0] < 0 || iq[0] >= nn[0] || iq[1] < 0 || iq[1] >= nn[1] ||
                        iq[2] < 0 || iq[2] >= nn[2]) continue;   /* outside Omega */
                    double W[3][3];
                    if (!bond_tensor(dim, ip, iq, h, M, alpha, n_infl, infl, W)) continue;
                    int64_t q = (iq[2] * nn[1] + iq[1]) * nn[0] + iq[0];
                    if (bond_broken(p, q, br_ptr, br_idx)) continue;  /* mu = 0 */
                    const double v = (nu && on_e) ? 0.5 * (nu[p] + nu[q]) : 1.0;
                    for (int a = 0; a < dim; ++a)
                        for (int b = 0; b < dim; ++b)
                            acc[a] += v * W[a][b] * (u[b * N + q] - u[b * N + p]);
                }
        for (int a = 0; a < dim; ++a) f[a * nrows + r] = acc[a];
    }
}

/*
 * Dense stiffness matrix A (dN x dN, row-major) of eq. (matrix) / (mae:e1):
 * off-diagonal blocks A_pq = mu_pq W_pq; diagonal block A_pp = -sum_q A_pq over
 * the same in-domain, unbroken neighbours (no Omega_c special-casing: every row
 * is built by the same rule; rows of constrained DOFs are the caller's to use
 * or ignore, Remark 1).  Row index = c*N + p.
 */
void oracle_assemble_dense(int dim, const int64_t *n, double h, int M, double alpha,
                           int n_infl, const double *infl,
                           const int64_t *br_ptr, const int64_t *br_idx, double *A)
{
    int64_t nn[3] = {n[0], n[1], dim == 3 ? n[2] : 1};
    int64_t N = nn[0] * nn[1] * nn[2];
    int64_t D = dim * N;
    int64_t Mz = dim == 3 ? M : 0;
    memset(A, 0, sizeof(double) * D * D);

#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        int64_t ip[3], iq[3];
        node_index(p, nn, ip);
        for (int64_t oz = -Mz; oz <= Mz; ++oz)
            for (int64_t oy = -M; oy <= M; ++oy)
                for (int64_t ox = -M; ox <= M; ++ox) {
                    iq[0] = ip[0] + ox; iq[1] = ip[1] + oy; iq[2] = ip[2] + oz;
                    if (iq[0] < 0 || iq[0] >= nn[0] || iq[1] < 0 || iq[1] >= nn[1] ||
                        iq[2] < 0 || iq[2] >= nn[2]) continue;
                    double W[3][3];
                    if (!bond_tensor(dim, ip, iq, h, M, alpha, n_infl, infl, W)) continue;
                    int64_t q = (iq[2] * nn[1] + iq[1]) * nn[0] + iq[0];
                    if (bond_broken(p, q, br_ptr, br_idx)) continue;
                    for (int a = 0; a < dim; ++a)
                        for (int b = 0; b < dim; ++b) {
                            A[(a * N + p) * D + (b * N + q)] = W[a][b];
                            A[(a * N + p) * D + (b * N + p)] -= W[a][b];
                        }
                }
    }
}
