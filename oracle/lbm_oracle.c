/*
 * lbm_oracle.c -- plain FP64 CPU oracle for the BGK lattice Boltzmann update with the
 * third-order anisotropic equilibrium of "Lattice Boltzmann Methods with Anisotropic
 * Equilibrium Distributions" (arXiv 2605.27004).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library. The HIP product path never links, loads or calls it, and the
 * two share no code, header, table or constant: every lattice quantity below is rebuilt here
 * from the paper's own recipe.
 *
 * Everything is IEEE double, built with -ffp-contract=off and without fast-math. The code is
 * deliberately literal and slow:
 *   - 1-D Gauss-Hermite rule: the nodes are the roots of H3(x) = x^3 - 3x and the weights
 *     come from w = n! / [n H2(x)]^2 with n = 3                               (App. C, eq:weights)
 *   - D2Q9 and D3Q27 are tensor products of that rule; D3Q19 is the subset |v|^2 <= 2 of
 *     D3Q27 with the weights fixed by the isotropy conditions (App. C, last paragraph)
 *   - lattice rescaling v = c/cs, u = s/cs: cs is the reciprocal of the outer node, so the
 *     outer nodes land on neighbouring lattice sites                            (Sec. 2.3)
 *   - K = A^-1 - I                                                                (eq:K-term)
 *   - Hermite tensors H2_ab = v_a v_b - d_ab, H3_abg = v_a v_b v_g - (v d + v d + v d)
 *     evaluated in lattice units                                        (eq:hermite_polynomials)
 *   - coefficients a2 = s s + cs^2 K, a3 = s s s + cs^2 (K s + K s + K s) and the discrete
 *     equilibrium f^eq_i as the explicit contraction of eq:3rd_order_equilibrium with the
 *     weights of eq:feq_i; order 2 drops the a3 term (the paper's comparison case, Sec. 4)
 *   - rho = sum_i f_i, rho s = sum_i f_i c_i                   (eq:a0discrete_f, eq:a1discrete_f)
 *   - collide then stream, dt = 1: f_i(t+1, x+c_i) = f_i + (f^eq_i - f_i)/tau     (eq:LBE_BGK)
 *     on a periodic Cartesian grid, written in push form into a second array.
 *
 * Population arrays are structure-of-arrays f[i][z][y][x] (x fastest) in THIS file's own
 * velocity order (the tensor-product enumeration below); callers map orders by velocity vector.
 *
 * Extensions beyond the paper (it names walls and forcing only as future work, Sec. 5); the
 * definitions below are the ones the library implements, written out plainly:
 *   - solid cells (mask = 1) carry no populations (kept at zero); a population leaving a fluid
 *     cell x towards a solid cell x + c_i returns to x in the opposite direction at the next
 *     step (halfway bounce-back): f_opp(i)(t+1, x) = f*_i(t, x);
 *   - gray cells (a fraction m in [0, 1] per cell, for differentiable obstacles): the
 *     post-collision populations are (1 - m) times the BGK result plus m times the cell's own
 *     pre-collision population of the opposite direction, f*_i = (1 - m) f^BGK_i + m f_opp(i),
 *     then streamed as usual (m = 1 reflects everything back on the node);
 *   - body force F (momentum per cell per step) by the exact-difference method:
 *     f*_i = f_i + (f^eq_i(rho, s) - f_i)/tau + [f^eq_i(rho, s + F/rho) - f^eq_i(rho, s)],
 *     with s = sum_i f_i c_i / rho, and the fluid velocity read out as (sum_i f_i c_i + F/2)/rho.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_D2Q9 0
#define ORC_D3Q19 1
#define ORC_D3Q27 2

#define ORC_TENSOR_THETA 0  /* T = cs^2 A^-1 (pressure tensor per unit density)        */
#define ORC_TENSOR_A 1      /* T = A of eq:equil, used as given                         */
#define ORC_TENSOR_ATILDE 2 /* T = A~ proportional to A; A = A~ / det(A~)^(1/d) (Sec. 4) */

#define QMAX 27

typedef struct {
    int d, q;
    int c[QMAX][3];   /* integer lattice velocities c_i                      */
    double w[QMAX];   /* quadrature weights w_i                              */
    double cs2;       /* lattice speed of sound squared                      */
    double H2[QMAX][3][3];
    double H3[QMAX][3][3][3];
} lattice_t;

/* ---- 1-D Gauss-Hermite rule with three nodes (App. C) -------------------------------- */


/* He3(x) = x^3 - 3x = x (x^2 - 3) has the roots x = 0 and x^2 = 3, i.e. 0 and +-sqrt(3)
 * (order 0, +, -). The weights depend on x only through x^2, so they are evaluated from the
 * exact squares rather than from a rounded sqrt(3). */
static const double GH_X2[3] = {0.0, 3.0, 3.0};
static const int GH_SIGN[3] = {0, 1, -1};

int orc_gh1d(double *nodes, double *weights)
{
    const int n = 3;
    for (int k = 0; k < n; ++k) {
        /* w_k = n! / [n He_{n-1}(x_k)]^2 (eq:weights), He_2(x) = x^2 - 1 */
        double nf = 6.0; /* 3! */
        double he2 = GH_X2[k] - 1.0;
        double den = (double)n * he2;
        nodes[k] = GH_SIGN[k] * sqrt(GH_X2[k]);
        weights[k] = nf / (den * den);
    }
    return 0;
}

static int build_lattice(int lattice, lattice_t *L)
{
    double x[3], w1[3];
    orc_gh1d(x, w1);
    /* v = c / cs with the outer node mapped to one lattice spacing: cs^2 = 1 / x_outer^2. */
    L->cs2 = 1.0 / GH_X2[1];
    int d = (lattice == ORC_D2Q9) ? 2 : 3;
    if (lattice != ORC_D2Q9 && lattice != ORC_D3Q19 && lattice != ORC_D3Q27) return -1;
    L->d = d;
    int q = 0;
    int nz = (d == 3) ? 3 : 1;
    for (int kz = 0; kz < nz; ++kz)
        for (int ky = 0; ky < 3; ++ky)
            for (int kx = 0; kx < 3; ++kx) {
                int k[3] = {kx, ky, (d == 3) ? kz : 0};
                int c[3] = {0, 0, 0};
                double w = 1.0;
                for (int a = 0; a < d; ++a) {
                    /* lattice velocity c = cs v = sign(v) sqrt(cs^2 v^2), an integer */
                    c[a] = GH_SIGN[k[a]] * (int)lround(sqrt(L->cs2 * GH_X2[k[a]]));
                    w *= w1[k[a]];
                }
                if (lattice == ORC_D3Q19) {
                    int n2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
                    if (n2 > 2) continue;
                    /* Weights of the reduced set from the isotropy conditions
                     * sum w = 1, sum w c_x^2 = cs^2, sum w c_x^2 c_y^2 = cs^4:
                     * rest 1/3, axis 1/18, edge 1/36. */
                    w = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
                }
                for (int a = 0; a < 3; ++a) L->c[q][a] = c[a];
                L->w[q] = w;
                ++q;
            }
    L->q = q;
    /* Hermite tensors in lattice units: H2 = c c - cs^2 d, H3 = c c c - cs^2 (c d + c d + c d)
     * (eq:hermite_polynomials with v = c/cs, multiplied through by cs^2 and cs^3). */
    for (int i = 0; i < q; ++i)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double dab = (a == b) ? 1.0 : 0.0;
                L->H2[i][a][b] = (double)L->c[i][a] * L->c[i][b] - L->cs2 * dab;
                for (int g = 0; g < 3; ++g) {
                    double dbg = (b == g) ? 1.0 : 0.0;
                    double dga = (g == a) ? 1.0 : 0.0;
                    L->H3[i][a][b][g] = (double)L->c[i][a] * L->c[i][b] * L->c[i][g]
                                      - L->cs2 * (L->c[i][a] * dbg + L->c[i][b] * dga + L->c[i][g] * dab);
                }
            }
    return 0;
}

int orc_lattice(int lattice, int *q, int *d, int *c, double *w, double *cs2)
{
    lattice_t L;
    if (build_lattice(lattice, &L)) return -1;
    if (q) *q = L.q;
    if (d) *d = L.d;
    if (cs2) *cs2 = L.cs2;
    for (int i = 0; i < L.q; ++i) {
        if (c)
            for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
        if (w) w[i] = L.w[i];
    }
    return 0;
}

/* ---- anisotropy tensor --------------------------------------------------------------- */

static double det_n(int d, const double *M)
{
    if (d == 2) return M[0] * M[3] - M[1] * M[2];
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6])
         + M[2] * (M[3] * M[7] - M[4] * M[6]);
}

/* Inverse by the adjugate: M^-1 = adj(M) / det(M). */
static int inv_n(int d, const double *M, double *R)
{
    double det = det_n(d, M);
    if (!(fabs(det) > 0.0)) return -1;
    if (d == 2) {
        R[0] = M[3] / det;
        R[1] = -M[1] / det;
        R[2] = -M[2] / det;
        R[3] = M[0] / det;
        return 0;
    }
    R[0] = (M[4] * M[8] - M[5] * M[7]) / det;
    R[1] = (M[2] * M[7] - M[1] * M[8]) / det;
    R[2] = (M[1] * M[5] - M[2] * M[4]) / det;
    R[3] = (M[5] * M[6] - M[3] * M[8]) / det;
    R[4] = (M[0] * M[8] - M[2] * M[6]) / det;
    R[5] = (M[2] * M[3] - M[0] * M[5]) / det;
    R[6] = (M[3] * M[7] - M[4] * M[6]) / det;
    R[7] = (M[1] * M[6] - M[0] * M[7]) / det;
    R[8] = (M[0] * M[4] - M[1] * M[3]) / det;
    return 0;
}

/* T is d x d row-major. Returns A^-1 (d x d row-major). */
int orc_tensor_to_ainv(int d, int kind, const double *T, double *Ainv)
{
    double cs2;
    lattice_t L;
    build_lattice(d == 2 ? ORC_D2Q9 : ORC_D3Q27, &L);
    cs2 = L.cs2;
    int n = d * d;
    if (kind == ORC_TENSOR_THETA) {
        /* second moment of f^eq is rho (cs^2 A^-1 + s s) (App. E): T/cs^2 = A^-1 */
        for (int k = 0; k < n; ++k) Ainv[k] = T[k] / cs2;
        return 0;
    }
    if (kind == ORC_TENSOR_A) return inv_n(d, T, Ainv);
    if (kind == ORC_TENSOR_ATILDE) {
        double det = det_n(d, T);
        if (!(det > 0.0)) return -1;
        double scale = pow(det, 1.0 / d);
        double A[9];
        for (int k = 0; k < n; ++k) A[k] = T[k] / scale;
        return inv_n(d, A, Ainv);
    }
    return -1;
}

/* ---- equilibrium ----------------------------------------------------------------------- */

/* f^eq_i for one cell. K is d x d row-major, s has d entries. */
static void feq_cell(const lattice_t *L, int order, const double K[3][3], double rho, const double s[3],
                     double *feq)
{
    const int d = L->d;
    const double cs2 = L->cs2;
    double a2[3][3], a3[3][3][3];
    /* App. B coefficients divided by rho, in lattice units (u = s/cs). */
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            a2[a][b] = s[a] * s[b] + cs2 * K[a][b];
            for (int g = 0; g < d; ++g)
                a3[a][b][g] = s[a] * s[b] * s[g] + cs2 * (K[a][b] * s[g] + K[b][g] * s[a] + K[g][a] * s[b]);
        }
    for (int i = 0; i < L->q; ++i) {
        double t1 = 0.0, t2 = 0.0, t3 = 0.0;
        for (int a = 0; a < d; ++a) t1 += L->c[i][a] * s[a];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) t2 += a2[a][b] * L->H2[i][a][b];
        if (order >= 3)
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b)
                    for (int g = 0; g < d; ++g) t3 += a3[a][b][g] * L->H3[i][a][b][g];
        double bracket = 1.0 + t1 / cs2 + t2 / (2.0 * cs2 * cs2) + t3 / (6.0 * cs2 * cs2 * cs2);
        feq[i] = L->w[i] * rho * bracket;
    }
}

static void k_from_ainv(int d, const double *Ainv, double K[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) K[a][b] = 0.0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) K[a][b] = Ainv[a * d + b] - ((a == b) ? 1.0 : 0.0); /* eq:K-term */
}

/* Ainv is d x d; s has d entries; feq has q entries. */
int orc_feq(int lattice, int order, const double *Ainv, double rho, const double *s, double *feq)
{
    lattice_t L;
    if (build_lattice(lattice, &L)) return -1;
    double K[3][3];
    k_from_ainv(L.d, Ainv, K);
    double sv[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < L.d; ++a) sv[a] = s[a];
    feq_cell(&L, order, K, rho, sv, feq);
    return 0;
}

/* ---- fields ---------------------------------------------------------------------------- */

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* f(0, x) = f^eq(rho0(x), s0(x)). rho0 is [N], s0 is [d][N], f is [q][N]. */
int orc_init_ext(int lattice, int order, int64_t nx, int64_t ny, int64_t nz, const double *Ainv, const double *rho0,
                 const double *s0, const uint8_t *mask, double *f, int nthreads)
{
    lattice_t L;
    if (build_lattice(lattice, &L)) return -1;
    double K[3][3];
    k_from_ainv(L.d, Ainv, K);
    const int64_t N = nx * ny * nz;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double s[3] = {0.0, 0.0, 0.0}, feq[QMAX];
        for (int a = 0; a < L.d; ++a) s[a] = s0[a * N + n];
        feq_cell(&L, order, K, rho0[n], s, feq);
        for (int i = 0; i < L.q; ++i) f[i * N + n] = (mask && mask[n]) ? 0.0 : feq[i];
    }
    return 0;
}

int orc_init(int lattice, int order, int64_t nx, int64_t ny, int64_t nz, const double *Ainv, const double *rho0,
             const double *s0, double *f, int nthreads)
{
    return orc_init_ext(lattice, order, nx, ny, nz, Ainv, rho0, s0, NULL, f, nthreads);
}

static int64_t wrap(int64_t v, int64_t n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

/* nsteps of eq:LBE_BGK on the periodic grid; f ([q][N]) holds the pre-collision state and
 * is advanced in place (a second array is allocated here). mask ([N], 1 = solid) and force
 * ([d]) may be NULL; see the header for their definitions. */
int orc_steps_gray(int lattice, int order, int64_t nx, int64_t ny, int64_t nz, const double *Ainv, double tau,
                   int64_t nsteps, double *f, const uint8_t *mask, const double *gray, const double *force,
                   int nthreads)
{
    lattice_t L;
    if (build_lattice(lattice, &L)) return -1;
    if (nx <= 0 || ny <= 0 || nz <= 0) return -1;
    double K[3][3];
    k_from_ainv(L.d, Ainv, K);
    const int64_t N = nx * ny * nz;
    const int q = L.q, d = L.d;
    int opp[QMAX];
    for (int i = 0; i < q; ++i)
        for (int k = 0; k < q; ++k)
            if (L.c[k][0] == -L.c[i][0] && L.c[k][1] == -L.c[i][1] && L.c[k][2] == -L.c[i][2]) opp[i] = k;
    double F[3] = {0.0, 0.0, 0.0};
    int forced = 0;
    if (force)
        for (int a = 0; a < d; ++a) {
            F[a] = force[a];
            if (F[a] != 0.0) forced = 1;
        }
    double *g = (double *)calloc((size_t)q * (size_t)N, sizeof(double));
    if (!g) return -2;
    set_threads(nthreads);
    double *cur = f, *nxt = g;
    for (int64_t t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static) collapse(2)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t n = (z * ny + y) * nx + x;
                    if (mask && mask[n]) {
                        for (int i = 0; i < q; ++i) nxt[i * N + n] = 0.0;
                        continue;
                    }
                    double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, s[3] = {0.0, 0.0, 0.0}, feq[QMAX], feqf[QMAX];
                    for (int i = 0; i < q; ++i) {
                        double fi = cur[i * N + n];
                        rho += fi;
                        for (int a = 0; a < d; ++a) j[a] += fi * L.c[i][a];
                    }
                    for (int a = 0; a < d; ++a) s[a] = j[a] / rho;
                    feq_cell(&L, order, K, rho, s, feq);
                    if (forced) {
                        double sf[3] = {0.0, 0.0, 0.0};
                        for (int a = 0; a < d; ++a) sf[a] = s[a] + F[a] / rho;
                        feq_cell(&L, order, K, rho, sf, feqf);
                    }
                    const double m = gray ? gray[n] : 0.0;
                    for (int i = 0; i < q; ++i) {
                        double fi = cur[i * N + n];
                        double post = fi + (feq[i] - fi) / tau;
                        if (forced) post += feqf[i] - feq[i];
                        if (gray) post = (1.0 - m) * post + m * cur[opp[i] * N + n];
                        int64_t xd = wrap(x + L.c[i][0], nx);
                        int64_t yd = wrap(y + L.c[i][1], ny);
                        int64_t zd = wrap(z + L.c[i][2], nz);
                        int64_t nd = (zd * ny + yd) * nx + xd;
                        if (mask && mask[nd])
                            nxt[opp[i] * N + n] = post; /* halfway bounce-back */
                        else
                            nxt[i * N + nd] = post;
                    }
                }
        double *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (cur != f) memcpy(f, cur, sizeof(double) * (size_t)q * (size_t)N);
    free(g);
    return 0;
}

int orc_steps_ext(int lattice, int order, int64_t nx, int64_t ny, int64_t nz, const double *Ainv, double tau,
                  int64_t nsteps, double *f, const uint8_t *mask, const double *force, int nthreads)
{
    return orc_steps_gray(lattice, order, nx, ny, nz, Ainv, tau, nsteps, f, mask, NULL, force, nthreads);
}

int orc_steps(int lattice, int order, int64_t nx, int64_t ny, int64_t nz, const double *Ainv, double tau,
              int64_t nsteps, double *f, int nthreads)
{
    return orc_steps_gray(lattice, order, nx, ny, nz, Ainv, tau, nsteps, f, NULL, NULL, NULL, nthreads);
}

/* rho = sum_i f_i, s = (sum_i f_i c_i + F/2) / rho (F = 0 when force is NULL); solid cells
 * (mask = 1) give rho = 0 and s = 0. rho is [N], s is [d][N]. */
int orc_moments_ext(int lattice, int64_t N, const double *f, const uint8_t *mask, const double *force, double *rho,
                    double *s)
{
    lattice_t L;
    if (build_lattice(lattice, &L)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        if (mask && mask[n]) {
            rho[n] = 0.0;
            for (int a = 0; a < L.d; ++a) s[a * N + n] = 0.0;
            continue;
        }
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < L.q; ++i) {
            double fi = f[i * N + n];
            r += fi;
            for (int a = 0; a < L.d; ++a) j[a] += fi * L.c[i][a];
        }
        rho[n] = r;
        for (int a = 0; a < L.d; ++a) s[a * N + n] = (j[a] + (force ? 0.5 * force[a] : 0.0)) / r;
    }
    return 0;
}

int orc_moments(int lattice, int64_t N, const double *f, double *rho, double *s)
{
    return orc_moments_ext(lattice, N, f, NULL, NULL, rho, s);
}

/* Objectives of the final state (used by gradient checks):
 *   kind 0: mass flux through the plane x = plane, sum over its cells of (j_x + F_x/2);
 *   kind 1: kinetic energy, sum over all cells of |j + F/2|^2 / (2 rho).
 * Solid cells of a binary mask are skipped. */
double orc_objective(int lattice, int64_t nx, int64_t ny, int64_t nz, const double *f, const uint8_t *mask,
                     const double *force, int kind, int64_t plane)
{
    lattice_t L;
    if (build_lattice(lattice, &L)) return NAN;
    const int64_t N = nx * ny * nz;
    double total = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        if (mask && mask[n]) continue;
        const int64_t x = n % nx;
        if (kind == 0 && x != plane) continue;
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < L.q; ++i) {
            double fi = f[i * N + n];
            r += fi;
            for (int a = 0; a < L.d; ++a) j[a] += fi * L.c[i][a];
        }
        for (int a = 0; a < L.d; ++a) j[a] += force ? 0.5 * force[a] : 0.0;
        if (kind == 0)
            total += j[0];
        else {
            double e = 0.0;
            for (int a = 0; a < L.d; ++a) e += j[a] * j[a];
            total += 0.5 * e / r;
        }
    }
    return total;
}
