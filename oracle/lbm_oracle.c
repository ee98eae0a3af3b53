/*
 * Plain FP64 CPU oracle for the D3Q19 BGK lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The HIP product path
 * never calls it, includes it or shares a table with it.
 *
 * Mawson & Revell, "Memory transfer optimization for a lattice Boltzmann
 * solver on Kepler architecture nVidia GPUs":
 *   - velocity set: Section 3.1, Eq. (4) (19 directions, i = 0..18)
 *   - weights and sound speed: text after Eq. (5)
 *   - BGK collision: Eqs. (2)-(3); equilibrium: Eq. (5)
 *   - moments: Eqs. (6)-(7)
 *   - fused pull iteration (stream from x - e_i, boundary conditions,
 *     moments, equilibrium, collision): Section 4.2, Algorithm 3
 *   - memory arrangement f[i*Nx*Ny*Nz + z*Ny*Nx + y*Nx + x]: Section 4.1
 *   - two copies of f swapped every step: Section 4.1 (footnote)
 *
 * Readings adopted where the paper is silent (it validates with on-site
 * velocity boundaries and uses no body force):
 *   - walls are halfway bounce-back on flagged solid cells; a moving wall adds
 *     6 w_i rho_w (e_i . u_w) with rho_w = 1 to the bounced population;
 *   - on-site velocity nodes (the boundary type of the paper's cavity
 *     validation, Section 5) are lattice nodes on the wall with a prescribed
 *     velocity; see onsite_node() below;
 *   - the body force follows Guo, Zheng & Shi (2002): u = (m + F/2)/rho and
 *     source (1 - 1/(2 tau)) w_i [3(e_i - u) + 9 (e_i . u) e_i] . F;
 *   - the box is periodic in x, y and z; walls exist only through flags;
 *   - the state is the post-collision population array.
 *
 * Everything is evaluated directly from the definitions, cell by cell, in
 * double precision, without blocking or algebraic rearrangement. Build with
 * -ffp-contract=off and without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* Eq. (4): columns of the 3x19 matrix, i = 0..18. */
static const int E[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 0, 1},  {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1},
};

/* Weights stated after Eq. (5): 1/3 for the rest direction, 1/18 for the six
 * axis directions, 1/36 for the twelve diagonal directions. */
static double weight(int i)
{
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* Opposite direction, found by search: the j with e_j = -e_i. */
static int opposite(int i)
{
    for (int j = 0; j < Q; ++j)
        if (E[j][0] == -E[i][0] && E[j][1] == -E[i][1] && E[j][2] == -E[i][2])
            return j;
    return -1;
}

static int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

static size_t cell_index(int x, int y, int z, int nx, int ny)
{
    /* Section 4.1: z*Ny*Nx + y*Nx + x */
    return ((size_t)z * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x;
}

/* ---------------------------------------------------------------------- */
/* Tables, exported so that tests can check them against Eq. (4).         */
/* ---------------------------------------------------------------------- */
void orc_tables(int* e_out /* 19*3 */, double* w_out /* 19 */, int* opp_out /* 19 */)
{
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) e_out[3 * i + a] = E[i][a];
        w_out[i] = weight(i);
        opp_out[i] = opposite(i);
    }
}

/* Eq. (5) with c_s^2 = 1/3: rho w_i [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u]. */
void orc_equilibrium(double rho, const double* u, double* feq)
{
    double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        feq[i] = rho * weight(i) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
    }
}

/* Moments of one cell's populations, Eqs. (6)-(7). */
static void moments(const double* p, double* rho, double* m)
{
    *rho = 0.0;
    m[0] = m[1] = m[2] = 0.0;
    for (int i = 0; i < Q; ++i) {
        *rho += p[i];
        for (int a = 0; a < 3; ++a) m[a] += E[i][a] * p[i];
    }
}

/* Guo source term for direction i (without the (1 - 1/(2 tau)) factor). */
static double guo_source(int i, const double* u, const double* F)
{
    double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
    double eF = E[i][0] * F[0] + E[i][1] * F[1] + E[i][2] * F[2];
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    return weight(i) * (3.0 * (eF - uF) + 9.0 * eu * eF);
}

/*
 * BGK collision of one cell (Eq. (3), the collision line of Algorithm 3)
 * with the Guo body force. p: pre-collision populations, s: result.
 */
void orc_collide_cell(const double* p, const double* F, double tau, double* s)
{
    double rho, m[3], u[3], feq[Q];
    moments(p, &rho, m);
    for (int a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * F[a]) / rho;
    orc_equilibrium(rho, u, feq);
    for (int i = 0; i < Q; ++i) {
        double G = guo_source(i, u, F);
        s[i] = p[i] - (p[i] - feq[i]) / tau + (1.0 - 1.0 / (2.0 * tau)) * G;
    }
}

/*
 * Explicit derivatives of the one-cell collision s = C(p; F, tau):
 *   J[i*19+j]  = ds_i/dp_j
 *   dF[i*3+b]  = ds_i/dF_b
 *   dtau[i]    = ds_i/dtau
 * Each entry is written as the chain rule through rho = sum p and
 * u = (m + F/2)/rho, term by term.
 */
void orc_collide_jacobian(const double* p, const double* F, double tau,
                          double* J, double* dF, double* dtau)
{
    double rho, m[3], u[3], feq[Q];
    double omega = 1.0 / tau;
    moments(p, &rho, m);
    for (int a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * F[a]) / rho;
    orc_equilibrium(rho, u, feq);

    double du_dp[3][Q]; /* du_a/dp_j = (e_ja - u_a)/rho */
    for (int a = 0; a < 3; ++a)
        for (int j = 0; j < Q; ++j) du_dp[a][j] = (E[j][a] - u[a]) / rho;

    for (int i = 0; i < Q; ++i) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        double eF = E[i][0] * F[0] + E[i][1] * F[1] + E[i][2] * F[2];
        double dfeq_drho = feq[i] / rho;
        double dfeq_du[3], dG_du[3], dG_dF[3];
        for (int a = 0; a < 3; ++a) {
            dfeq_du[a] = rho * weight(i) * (3.0 * E[i][a] + 9.0 * eu * E[i][a] - 3.0 * u[a]);
            dG_du[a] = weight(i) * (-3.0 * F[a] + 9.0 * E[i][a] * eF);
            dG_dF[a] = weight(i) * (3.0 * (E[i][a] - u[a]) + 9.0 * eu * E[i][a]);
        }
        for (int j = 0; j < Q; ++j) {
            double dfeq_dpj = dfeq_drho;
            double dG_dpj = 0.0;
            for (int a = 0; a < 3; ++a) {
                dfeq_dpj += dfeq_du[a] * du_dp[a][j];
                dG_dpj += dG_du[a] * du_dp[a][j];
            }
            J[i * Q + j] = (i == j ? 1.0 - omega : 0.0) + omega * dfeq_dpj
                           + (1.0 - 0.5 * omega) * dG_dpj;
        }
        for (int b = 0; b < 3; ++b) {
            double du_dFb = 0.5 / rho; /* du_b/dF_b; other components 0 */
            dF[i * 3 + b] = omega * dfeq_du[b] * du_dFb
                            + (1.0 - 0.5 * omega) * (dG_du[b] * du_dFb + dG_dF[b]);
        }
        double G = guo_source(i, u, F);
        dtau[i] = ((p[i] - feq[i]) + 0.5 * G) / (tau * tau);
    }
}

/* Force at cell c: field (SoA [3][N]) if given, else uniform, else zero. */
static void force_at(const double* field, const double* uniform, size_t N, size_t c, double* F)
{
    for (int a = 0; a < 3; ++a) {
        if (field) F[a] = field[(size_t)a * N + c];
        else if (uniform) F[a] = uniform[a];
        else F[a] = 0.0;
    }
}

/*
 * Cell types: 0 fluid, 1 wall, 2 wall moving with u_w, 3 on-site velocity
 * node at rest, 4 on-site velocity node moving with u_w. Types 1 and 2 are
 * solid; types 0, 3 and 4 are fluid nodes that stream and collide.
 */
static int flag_at(const uint8_t* flags, size_t c) { return flags ? flags[c] : 0; }
static int is_solid(int fl) { return fl == 1 || fl == 2; }
static int is_onsite(int fl) { return fl == 3 || fl == 4; }

/*
 * Pull gather for fluid cell (x,y,z): p_i = s_i(x - e_i), or, when x - e_i is
 * solid, the bounced population s_opp(i)(x) plus the moving-wall term.
 * with_wall_term = 0 leaves the moving-wall term out (pure permutation).
 */
static void pull(int nx, int ny, int nz, const uint8_t* flags, const double* uw,
                 int with_wall_term, const double* s, int x, int y, int z, double* p)
{
    size_t N = (size_t)nx * ny * nz;
    size_t c = cell_index(x, y, z, nx, ny);
    for (int i = 0; i < Q; ++i) {
        int xs = wrap(x - E[i][0], nx), ys = wrap(y - E[i][1], ny), zs = wrap(z - E[i][2], nz);
        size_t src = cell_index(xs, ys, zs, nx, ny);
        int fl = flag_at(flags, src);
        if (!is_solid(fl)) {
            p[i] = s[(size_t)i * N + src];
        } else {
            p[i] = s[(size_t)opposite(i) * N + c];
            if (fl == 2 && with_wall_term && uw) {
                double eu = E[i][0] * uw[0] + E[i][1] * uw[1] + E[i][2] * uw[2];
                p[i] += 6.0 * weight(i) * 1.0 * eu; /* rho_w = 1 */
            }
        }
    }
}

/* Solve the 4x4 system A z = r by Gaussian elimination with partial
 * pivoting. Returns -1 when a pivot vanishes. */
static int solve4(double A[4][4], double r[4], double z[4])
{
    for (int k = 0; k < 4; ++k) {
        int piv = k;
        for (int i = k + 1; i < 4; ++i)
            if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
        if (fabs(A[piv][k]) < 1e-300) return -1;
        if (piv != k) {
            for (int j = 0; j < 4; ++j) {
                double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t;
            }
            double t = r[k]; r[k] = r[piv]; r[piv] = t;
        }
        for (int i = k + 1; i < 4; ++i) {
            double f = A[i][k] / A[k][k];
            for (int j = k; j < 4; ++j) A[i][j] -= f * A[k][j];
            r[i] -= f * r[k];
        }
    }
    for (int k = 3; k >= 0; --k) {
        double v = r[k];
        for (int j = k + 1; j < 4; ++j) v -= A[k][j] * z[j];
        z[k] = v / A[k][k];
    }
    return 0;
}

/*
 * On-site velocity node (the boundary condition family the paper validates
 * with, Section 5, after Hecht & Harting). The node sits on the wall and its
 * velocity u is prescribed. After the pull, the populations that would have
 * come from solid cells (unknown[i] != 0) are missing and are rebuilt here.
 * The paper prints no formulas; the reading adopted:
 *   - an unknown direction i whose opposite is known takes the opposite's
 *     value plus the equilibrium difference and a transverse correction:
 *       p_i = p_opp(i) + 6 w_i e_i . j + e_i . lambda,   j = rho u - F/2
 *     (j is the bare momentum that gives velocity u once the Guo term F/2 is
 *     added in the collision);
 *   - when both i and opp(i) are unknown (edges and corners of a box), the
 *     pair takes the equilibrium at (rho, u), split so that it carries the
 *     same bare momentum: p_i = f^eq_i(rho, u) - (3/2) w_i e_i . F;
 *   - rho and lambda are whatever makes the node carry mass rho and bare
 *     momentum j: sum_i p_i = rho and sum_i e_i p_i = j.
 * The populations are affine in z = (rho, lambda_x, lambda_y, lambda_z), so
 * the four conditions form a 4x4 linear system, solved directly.
 * Returns -1 if the system is singular.
 */
static int onsite_node(double* p, const int* unknown, const double* u, const double* F)
{
    double base[Q], coef[Q][4];
    for (int i = 0; i < Q; ++i) {
        for (int k = 0; k < 4; ++k) coef[i][k] = 0.0;
        base[i] = p[i];
        if (!unknown[i]) continue;
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        double eF = E[i][0] * F[0] + E[i][1] * F[1] + E[i][2] * F[2];
        int o = opposite(i);
        if (!unknown[o]) {
            /* p_opp + 6 w_i e_i.(rho u - F/2) + e_i.lambda */
            base[i] = p[o] - 3.0 * weight(i) * eF;
            coef[i][0] = 6.0 * weight(i) * eu;
            for (int a = 0; a < 3; ++a) coef[i][1 + a] = E[i][a];
        } else {
            /* rho w_i (1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u) - 1.5 w_i e_i.F */
            double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            base[i] = -1.5 * weight(i) * eF;
            coef[i][0] = weight(i) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
        }
    }
    /* row 0: sum p - rho = 0; row 1+a: sum e_a p - (rho u_a - F_a/2) = 0 */
    double A[4][4], r[4], z[4];
    for (int row = 0; row < 4; ++row) {
        double rb = 0.0;
        for (int k = 0; k < 4; ++k) A[row][k] = 0.0;
        for (int i = 0; i < Q; ++i) {
            double m = row == 0 ? 1.0 : (double)E[i][row - 1];
            rb += m * base[i];
            for (int k = 0; k < 4; ++k) A[row][k] += m * coef[i][k];
        }
        if (row == 0) {
            A[0][0] -= 1.0;
            r[0] = -rb;
        } else {
            A[row][0] -= u[row - 1];
            r[row] = -(rb + 0.5 * F[row - 1]);
        }
    }
    if (solve4(A, r, z) != 0) return -1;
    for (int i = 0; i < Q; ++i) {
        if (!unknown[i]) continue;
        double v = base[i];
        for (int k = 0; k < 4; ++k) v += coef[i][k] * z[k];
        p[i] = v;
    }
    return 0;
}

/*
 * One fused pull iteration (Algorithm 3) over the whole box.
 * collide = 0 gives streaming with bounce-back only (no moving-wall term, and
 * on-site nodes treated as ordinary fluid nodes): an exact permutation of the
 * fluid populations.
 * Solid cells are copied unchanged. Returns 0, -1 on a bad flag value, -3
 * when an on-site node's conditions cannot be solved.
 */
int orc_step(int nx, int ny, int nz, const uint8_t* flags, double tau, const double* uw,
             const double* force_field, const double* force_uniform, int collide,
             const double* s_in, double* s_out)
{
    size_t N = (size_t)nx * ny * nz;
    int bad = 0;
    if (flags)
        for (size_t c = 0; c < N; ++c)
            if (flags[c] > 4) return -1;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                size_t c = cell_index(x, y, z, nx, ny);
                int fl = flag_at(flags, c);
                if (is_solid(fl)) {
                    for (int i = 0; i < Q; ++i) s_out[(size_t)i * N + c] = s_in[(size_t)i * N + c];
                    continue;
                }
                double p[Q], s[Q], F[3];
                pull(nx, ny, nz, flags, uw, collide, s_in, x, y, z, p);
                if (collide) {
                    force_at(force_field, force_uniform, N, c, F);
                    if (is_onsite(fl)) {
                        int unknown[Q];
                        double un[3] = {0.0, 0.0, 0.0};
                        for (int i = 0; i < Q; ++i) {
                            size_t src = cell_index(wrap(x - E[i][0], nx), wrap(y - E[i][1], ny),
                                                    wrap(z - E[i][2], nz), nx, ny);
                            unknown[i] = is_solid(flag_at(flags, src));
                        }
                        if (fl == 4 && uw)
                            for (int a = 0; a < 3; ++a) un[a] = uw[a];
                        if (onsite_node(p, unknown, un, F) != 0) bad = 1;
                    }
                    orc_collide_cell(p, F, tau, s);
                } else {
                    for (int i = 0; i < Q; ++i) s[i] = p[i];
                }
                for (int i = 0; i < Q; ++i) s_out[(size_t)i * N + c] = s[i];
            }
        }
    }
    return bad ? -3 : 0;
}

/* n steps in place on s (uses one scratch copy). Returns 0, -1 bad flags, -2 OOM. */
int orc_run(int nx, int ny, int nz, const uint8_t* flags, double tau, const double* uw,
            const double* force_field, const double* force_uniform, int collide, int nsteps,
            double* s)
{
    size_t N = (size_t)nx * ny * nz;
    double* tmp = (double*)malloc(sizeof(double) * Q * N);
    if (!tmp) return -2;
    int rc = 0;
    double *a = s, *b = tmp;   /* the two copies of Section 4.1, swapped every step */
    for (int t = 0; t < nsteps && rc == 0; ++t) {
        rc = orc_step(nx, ny, nz, flags, tau, uw, force_field, force_uniform, collide, a, b);
        double* c = a; a = b; b = c;
    }
    if (a != s) memcpy(s, a, sizeof(double) * Q * N);
    free(tmp);
    return rc;
}

/*
 * Macroscopic fields of a post-collision state (Eqs. (6)-(7)): rho = sum s_i,
 * u = (sum e_i s_i - F/2)/rho. The Guo collision adds F to the momentum of a
 * cell, so this equals the velocity used inside the collision. Solid cells
 * report rho = 0 and u = 0. rho: [N], u: [3][N].
 */
void orc_macros(int nx, int ny, int nz, const uint8_t* flags, const double* force_field,
                const double* force_uniform, const double* s, double* rho, double* u)
{
    size_t N = (size_t)nx * ny * nz;
    for (size_t c = 0; c < N; ++c) {
        if (is_solid(flag_at(flags, c))) {
            rho[c] = 0.0;
            u[c] = u[N + c] = u[2 * N + c] = 0.0;
            continue;
        }
        double p[Q], r, m[3], F[3];
        for (int i = 0; i < Q; ++i) p[i] = s[(size_t)i * N + c];
        moments(p, &r, m);
        force_at(force_field, force_uniform, N, c, F);
        rho[c] = r;
        for (int a = 0; a < 3; ++a) u[(size_t)a * N + c] = (m[a] - 0.5 * F[a]) / r;
    }
}

/* f = f^eq(rho, u) per cell; rho NULL means 1, u NULL means 0. f: [19][N]. */
void orc_init_equilibrium(size_t N, const double* rho, const double* u, double* f)
{
    for (size_t c = 0; c < N; ++c) {
        double r = rho ? rho[c] : 1.0;
        double uc[3] = {0.0, 0.0, 0.0};
        if (u)
            for (int a = 0; a < 3; ++a) uc[a] = u[(size_t)a * N + c];
        double feq[Q];
        orc_equilibrium(r, uc, feq);
        for (int i = 0; i < Q; ++i) f[(size_t)i * N + c] = feq[i];
    }
}

/* ---------------------------------------------------------------------- */
/* Storage rounding used to model 16-bit offset storage.                   */
/* ---------------------------------------------------------------------- */

/*
 * Round a double to the nearest value with `mant` explicit mantissa bits and
 * minimum normal exponent emin (IEEE-style gradual underflow below it),
 * ties to even. Overflow is not handled: offsets are far below the maximum
 * of either format. binary16: mant = 10, emin = -14. bfloat16: mant = 7,
 * emin = -126.
 */
static double round_to_format(double v, int mant, int emin)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    frexp(fabs(v), &e);          /* |v| = m * 2^e with m in [0.5, 1) */
    int exp_unbiased = e - 1;    /* |v| = 1.xxx * 2^exp_unbiased */
    if (exp_unbiased < emin) exp_unbiased = emin;
    double quantum = ldexp(1.0, exp_unbiased - mant);
    double q = v / quantum;      /* exact: scaling by a power of two */
    double r = nearbyint(q);     /* default rounding mode: nearest, ties even */
    return r * quantum;
}

double orc_round_half(double v) { return round_to_format(v, 10, -14); }
double orc_round_bf16(double v) { return round_to_format(v, 7, -126); }

/*
 * Model of offset storage: f_i -> w_i + round(f_i - w_i) in the given format
 * (1 = binary16, 2 = bfloat16, 0 = float32 of the plain value), element-wise
 * over a [19][N] array. The offset f_i - w_i is formed in double.
 */
void orc_quantize(size_t N, int format, const double* f, double* out)
{
    for (int i = 0; i < Q; ++i) {
        double w = weight(i);
        for (size_t c = 0; c < N; ++c) {
            double v = f[(size_t)i * N + c];
            double r;
            if (format == 1) r = w + orc_round_half(v - w);
            else if (format == 2) r = w + orc_round_bf16(v - w);
            else r = (double)(float)v;
            out[(size_t)i * N + c] = r;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Discrete adjoint of the rollout (not in the paper; discretise then       */
/* differentiate the recurrence above).                                     */
/* ---------------------------------------------------------------------- */

/*
 * Gradient of a loss L(u(T)) with respect to the force field and tau, where
 * u(T) is the macroscopic velocity of the state after T steps from s0.
 * g = dL/du(T) as [3][N] (zero at solid cells). All T+1 states are kept.
 * For each step, the 19x19 collision Jacobian of every fluid cell is formed
 * explicitly and multiplied plainly; streaming is transposed link by link.
 * grad_F: [3][N] out; *grad_tau out. Returns 0, -1 when the lattice has
 * on-site velocity nodes (not covered by this adjoint), or -2 on allocation
 * failure.
 */
int orc_adjoint(int nx, int ny, int nz, const uint8_t* flags, double tau, const double* uw,
                const double* force_field, const double* s0, int T, const double* g,
                double* grad_F, double* grad_tau)
{
    size_t N = (size_t)nx * ny * nz;
    size_t SZ = (size_t)Q * N;
    if (flags)
        for (size_t c = 0; c < N; ++c)
            if (flags[c] > 2) return -1;
    double* states = (double*)malloc(sizeof(double) * SZ * (size_t)(T + 1));
    double* a = (double*)malloc(sizeof(double) * SZ);
    double* b = (double*)malloc(sizeof(double) * SZ);
    double* zero_force = (double*)calloc(3 * N, sizeof(double));
    double* tau_part = (double*)calloc((size_t)nz, sizeof(double));
    if (!states || !a || !b || !zero_force || !tau_part) {
        free(states); free(a); free(b); free(zero_force); free(tau_part);
        return -2;
    }
    const double* Ff = force_field ? force_field : zero_force;

    memcpy(states, s0, sizeof(double) * SZ);
    for (int t = 0; t < T; ++t)
        orc_step(nx, ny, nz, flags, tau, uw, Ff, NULL, 1, states + SZ * t, states + SZ * (t + 1));

    /* Seed: a_j = dL/ds_j(T) = sum_a g_a du_a/ds_j with du_a/ds_j = (e_ja - u_a)/rho
     * for u = (m - F/2)/rho; direct term dL/dF_a = -g_a / (2 rho). */
    const double* sT = states + SZ * T;
    for (size_t c = 0; c < N; ++c) {
        for (int i = 0; i < Q; ++i) a[(size_t)i * N + c] = 0.0;
        for (int k = 0; k < 3; ++k) grad_F[(size_t)k * N + c] = 0.0;
        if (flag_at(flags, c) != 0) continue;
        double p[Q], r, m[3], u[3];
        for (int i = 0; i < Q; ++i) p[i] = sT[(size_t)i * N + c];
        moments(p, &r, m);
        for (int k = 0; k < 3; ++k) u[k] = (m[k] - 0.5 * Ff[(size_t)k * N + c]) / r;
        for (int j = 0; j < Q; ++j) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v += g[(size_t)k * N + c] * (E[j][k] - u[k]) / r;
            a[(size_t)j * N + c] = v;
        }
        for (int k = 0; k < 3; ++k) grad_F[(size_t)k * N + c] = -g[(size_t)k * N + c] / (2.0 * r);
    }

    for (int t = T - 1; t >= 0; --t) {
        const double* st = states + SZ * t;
        /* b = J_C(p^t)^T a per fluid cell; accumulate dF and dtau terms. */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z) {
            double part = 0.0;
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t c = cell_index(x, y, z, nx, ny);
                    for (int i = 0; i < Q; ++i) b[(size_t)i * N + c] = 0.0;
                    if (flag_at(flags, c) != 0) continue;
                    double p[Q], F[3], J[Q * Q], dF[Q * 3], dtau[Q], ac[Q];
                    pull(nx, ny, nz, flags, uw, 1, st, x, y, z, p);
                    force_at(Ff, NULL, N, c, F);
                    orc_collide_jacobian(p, F, tau, J, dF, dtau);
                    for (int i = 0; i < Q; ++i) ac[i] = a[(size_t)i * N + c];
                    for (int j = 0; j < Q; ++j) {
                        double v = 0.0;
                        for (int i = 0; i < Q; ++i) v += ac[i] * J[i * Q + j];
                        b[(size_t)j * N + c] = v;
                    }
                    for (int k = 0; k < 3; ++k) {
                        double v = 0.0;
                        for (int i = 0; i < Q; ++i) v += ac[i] * dF[i * 3 + k];
                        grad_F[(size_t)k * N + c] += v;
                    }
                    for (int i = 0; i < Q; ++i) part += ac[i] * dtau[i];
                }
            tau_part[z] += part;
        }
        /* a = P^T b: for fluid y, a_j(y) = b_j(y + e_j) if y + e_j is fluid,
         * else b_opp(j)(y) (the bounced link). Solid cells get 0. */
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t c = cell_index(x, y, z, nx, ny);
                    for (int j = 0; j < Q; ++j) {
                        double v = 0.0;
                        if (flag_at(flags, c) == 0) {
                            size_t d = cell_index(wrap(x + E[j][0], nx), wrap(y + E[j][1], ny),
                                                  wrap(z + E[j][2], nz), nx, ny);
                            if (flag_at(flags, d) == 0) v = b[(size_t)j * N + d];
                            else v = b[(size_t)opposite(j) * N + c];
                        }
                        a[(size_t)j * N + c] = v;
                    }
                }
    }
    double gt = 0.0;
    for (int z = 0; z < nz; ++z) gt += tau_part[z];
    *grad_tau = gt;

    free(states); free(a); free(b); free(zero_force); free(tau_part);
    return 0;
}

/* Number of OpenMP threads the loops above use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads of later calls (no effect without OpenMP). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
