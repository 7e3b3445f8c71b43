/*
 * lbm_oracle.c -- plain, slow, FP64 reference of the D3Q19 node update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, table or header with the GPU
 * path.
 *
 * What it computes (Wittmann, Zeiser, Hager, Wellein, "Comparison of
 * different Propagation Steps for the Lattice Boltzmann Method"):
 *
 *   - the two-step two-grid algorithm of Sec. 2: a collision loop that reads
 *     lattice A and stores the post-collision values at the same node of
 *     lattice B, then a separate propagation loop that moves them from B back
 *     to the neighbours in A (Sec. 2, Table 1);
 *   - the propagation is written in "pull" form (Sec. 3, Fig. 1(c)):
 *         A[i][x] = B[i][x - c_i]
 *     with half-way bounce-back A[i][x] = B[opp(i)][x] when x - c_i is solid
 *     or lies outside a non-periodic axis;
 *   - the collision is single-relaxation-time BGK with the Guo, Zheng & Shi
 *     (2002) body-force term, or the two-relaxation-time (TRT) collision the
 *     paper's own solver uses (Sec. 10, ref. [15]) with the same force term
 *     split into even and odd parts.  The paper prints no operator; these are
 *     the readings taken.
 *   - open boundaries (velocity and pressure in-/outlets, Sec. 6) as link
 *     rules on the bounced population, see boundary_value();
 *   - the index array of indirect addressing (Sec. 1): fluid nodes numbered
 *     in lexicographic order (x fastest), IDX[k][n] = id of the neighbour in
 *     direction c_{k+1}, -1 when that neighbour is solid.
 *
 * Storage: f[i*ncell + cell], cell = x + nx*(y + ny*z); solid[cell] = 1 for
 * solid cells.  Solid cells are never updated and never read as sources.
 *
 * Optional storage rounding ("quant") mimics the reduced-precision storage
 * forms: 1 = each stored value rounded to binary32; 2 = the shifted deviation
 * (f_i - w_i)*sigma rounded to binary16; 3 = that deviation rounded to
 * binary32 (IEEE 754 round-to-nearest-even throughout).
 * The arithmetic itself is always FP64.
 *
 * Parity pins for every function here live in tests/test_oracle.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* D3Q19 velocity set: rest, 6 axis neighbours, 12 edge (diagonal)
 * neighbours.  Order: each direction is followed by its opposite. */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0},
    {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0},
    {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1},
    {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1},
    {0, 1, -1}, {0, -1, 1},
};

/* Weights: 1/3 rest, 1/18 axis, 1/36 edge. */
static double WV[Q];
static int OPPV[Q];
static int tables_ready = 0;

static void init_tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < Q; ++i) {
        int n2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
        WV[i] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        /* opposite: the direction with c_j = -c_i, found by search */
        for (int j = 0; j < Q; ++j)
            if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2])
                OPPV[i] = j;
    }
    tables_ready = 1;
}

void ora_tables(int *c_out, double *w_out, int *opp_out)
{
    init_tables();
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) c_out[3 * i + a] = CV[i][a];
        w_out[i] = WV[i];
        opp_out[i] = OPPV[i];
    }
}

/* Second-order equilibrium, c_s^2 = 1/3:
 *   f_i^eq = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u)                 */
void ora_equilibrium(double rho, const double u[3], double feq[Q])
{
    init_tables();
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        feq[i] = WV[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Guo forcing term for force density F = rho g:
 *   S_i = (1 - omega/2) w_i [ 3 (c_i - u) + 9 (c_i.u) c_i ] . F          */
void ora_guo_source(double rho, const double u[3], double omega, const double g[3], double S[Q])
{
    init_tables();
    double F[3] = {rho * g[0], rho * g[1], rho * g[2]};
    for (int i = 0; i < Q; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
            s += (3.0 * (CV[i][a] - u[a]) + 9.0 * cu * CV[i][a]) * F[a];
        S[i] = (1.0 - 0.5 * omega) * WV[i] * s;
    }
}

/* TRT (Ginzburg): split each pair of opposite directions i, i' into even and
 * odd parts a^+ = (a_i + a_i')/2, a^- = (a_i - a_i')/2 and relax them with w+
 * and w-; the Guo source S (computed with omega = 0, i.e. without its
 * prefactor) gets (1 - w+/2) on its even and (1 - w-/2) on its odd part. */
void ora_collide_node_trt(const double f[Q], double wp, double wm, const double g[3], double out[Q])
{
    init_tables();
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * f[i];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * rho * g[a]) / rho;
    double feq[Q], S[Q];
    ora_equilibrium(rho, u, feq);
    ora_guo_source(rho, u, 0.0, g, S);
    for (int i = 0; i < Q; ++i) {
        int o = OPPV[i];
        double fp = 0.5 * (f[i] + f[o]), fm = 0.5 * (f[i] - f[o]);
        double ep = 0.5 * (feq[i] + feq[o]), em = 0.5 * (feq[i] - feq[o]);
        double sp = 0.5 * (S[i] + S[o]), sm = 0.5 * (S[i] - S[o]);
        out[i] = f[i] - wp * (fp - ep) - wm * (fm - em) + (1.0 - 0.5 * wp) * sp + (1.0 - 0.5 * wm) * sm;
    }
}

/* One node: collider 1 = BGK + Guo, 0 = identity (stream-only runs). */
void ora_collide_node(const double f[Q], double omega, const double g[3], int collider, double out[Q])
{
    init_tables();
    if (collider == 0) {
        for (int i = 0; i < Q; ++i) out[i] = f[i];
        return;
    }
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * f[i];
    }
    /* physical velocity carries half the force impulse */
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * rho * g[a]) / rho;
    double feq[Q], S[Q];
    ora_equilibrium(rho, u, feq);
    ora_guo_source(rho, u, omega, g, S);
    for (int i = 0; i < Q; ++i) out[i] = f[i] - omega * (f[i] - feq[i]) + S[i];
}

/* Nearest binary16 value (round to nearest, ties to even), returned as a
 * double.  Written from the IEEE 754 binary16 format: 11 significant bits,
 * exponent range [-14, 15], subnormal quantum 2^-24, overflow to infinity. */
double ora_round_half(double v)
{
    if (isnan(v) || isinf(v) || v == 0.0) return v;
    double a = fabs(v);
    int e;
    frexp(a, &e);          /* a in [2^(e-1), 2^e) */
    int ex = e - 1;
    if (ex < -14) ex = -14; /* subnormal range has a fixed quantum */
    double quantum = ldexp(1.0, ex - 10);
    double r = nearbyint(a / quantum) * quantum;
    if (r >= 65536.0) r = INFINITY;
    return copysign(r, v);
}

void ora_round_half_array(const double *in, double *out, long n)
{
    for (long k = 0; k < n; ++k) out[k] = ora_round_half(in[k]);
}

static double quantize_value(double v, int i, int quant, double sigma)
{
    if (quant == 1) return (double)(float)v;
    if (quant == 2) return WV[i] + ora_round_half((v - WV[i]) * sigma) / sigma;
    if (quant == 3) return WV[i] + (double)(float)((v - WV[i]) * sigma) / sigma;
    return v;
}

static int resolve_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Round every stored value of the fluid cells to the storage precision. */
void ora_quantize_field(double *A, const uint8_t *solid, const int dims[3], int quant, double sigma)
{
    init_tables();
    long ncell = (long)dims[0] * dims[1] * dims[2];
    for (long c = 0; c < ncell; ++c) {
        if (solid[c]) continue;
        for (int i = 0; i < Q; ++i) A[i * ncell + c] = quantize_value(A[i * ncell + c], i, quant, sigma);
    }
}

/* Collision loop of the two-step algorithm: A -> B at the same location. */
void ora_collide(const double *A, double *B, const uint8_t *solid, const int dims[3], double omega,
                 double omega_minus, const double g[3], int collider, int quant, double sigma, int nthreads)
{
    init_tables();
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const long ncell = (long)nx * ny * nz;
    int nt = resolve_threads(nthreads);
    (void)nt;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                long c = x + (long)nx * (y + (long)ny * z);
                if (solid[c]) continue;
                double f[Q], fs[Q];
                for (int i = 0; i < Q; ++i) f[i] = A[i * ncell + c];
                if (collider == 2)
                    ora_collide_node_trt(f, omega, omega_minus, g, fs);
                else
                    ora_collide_node(f, omega, g, collider, fs);
                for (int i = 0; i < Q; ++i) B[i * ncell + c] = quantize_value(fs[i], i, quant, sigma);
            }
        }
    }
}

/* Source cell of a pull along direction i: x - c_i.  Returns -1 when that
 * cell is outside a non-periodic axis. */
static long pull_source(int x, int y, int z, int i, const int dims[3], const int periodic[3])
{
    int p[3] = {x - CV[i][0], y - CV[i][1], z - CV[i][2]};
    for (int a = 0; a < 3; ++a) {
        if (p[a] < 0 || p[a] >= dims[a]) {
            if (!periodic[a]) return -1;
            p[a] = (p[a] + dims[a]) % dims[a];
        }
    }
    return p[0] + (long)dims[0] * (p[1] + (long)dims[1] * p[2]);
}

/* Propagation loop of the two-step algorithm (pull form), B -> A. */
/* Open boundaries (the in-/outlet routines the AA pattern needs in both
 * parities, Sec. 6).  A non-fluid cell with mask value m >= 2 belongs to
 * boundary class m - 1 (m <= 5; larger values are walls);
 * bc[5 (m - 2) + 0..4] = {kind, rho, ux, uy, uz}:
 *   kind 0  wall: plain half-way bounce-back;
 *   kind 1  velocity boundary, a wall moving with u (Ladd 1994): the
 *           bounced population gains the momentum the moving wall imparts,
 *             f_i(x, t+1) = f*_opp(i)(x, t) + 6 w_i rho c_i.u ;
 *   kind 2  pressure boundary of density rho and velocity u, by
 *           anti-bounce-back:
 *             f_i(x, t+1) = -f*_opp(i)(x, t) + 2 w_i rho (1 + 9/2 (c_i.u)^2 - 3/2 u.u).
 * Mask value 1, cells outside a non-periodic axis, and bc == NULL are plain
 * walls.  `bounced` is f*_opp(i)(x, t), i the direction that arrives at x. */
static double boundary_value(double bounced, int i, int m, const double *bc)
{
    if (m < 2 || m > 5 || !bc) return bounced;
    const double *e = bc + 5 * (m - 2);
    const int kind = (int)e[0];
    const double rho = e[1];
    const double cu = CV[i][0] * e[2] + CV[i][1] * e[3] + CV[i][2] * e[4];
    const double uu = e[2] * e[2] + e[3] * e[3] + e[4] * e[4];
    if (kind == 1) return bounced + 6.0 * WV[i] * rho * cu;
    if (kind == 2) return -bounced + 2.0 * WV[i] * rho * (1.0 + 4.5 * cu * cu - 1.5 * uu);
    return bounced;
}

void ora_stream(const double *B, double *A, const uint8_t *solid, const int dims[3], const int periodic[3],
                const double *bc, int nthreads)
{
    init_tables();
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const long ncell = (long)nx * ny * nz;
    int nt = resolve_threads(nthreads);
    (void)nt;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                long c = x + (long)nx * (y + (long)ny * z);
                if (solid[c]) continue;
                for (int i = 0; i < Q; ++i) {
                    long s = pull_source(x, y, z, i, dims, periodic);
                    if (s < 0 || solid[s]) /* half-way bounce-back, or an open boundary */
                        A[i * ncell + c] = boundary_value(B[OPPV[i] * ncell + c], i, s < 0 ? 1 : solid[s], bc);
                    else
                        A[i * ncell + c] = B[i * ncell + s];
                }
            }
        }
    }
}

/* nsteps full time steps of the two-step algorithm; A holds f(t) before and
 * f(t + nsteps) after; B is the intermediate lattice. */
void ora_run_ts(double *A, double *B, const uint8_t *solid, const int dims[3], const int periodic[3],
                double omega, double omega_minus, const double g[3], int collider, int quant, double sigma,
                const double *bc, long nsteps, int nthreads)
{
    for (long t = 0; t < nsteps; ++t) {
        ora_collide(A, B, solid, dims, omega, omega_minus, g, collider, quant, sigma, nthreads);
        ora_stream(B, A, solid, dims, periodic, bc, nthreads);
    }
}

/* Total mass M = sum rho and raw momentum J = sum_x sum_i c_i f_i over the
 * fluid cells, summed serially in lexicographic order. */
void ora_moments(const double *A, const uint8_t *solid, const int dims[3], double out[4])
{
    init_tables();
    const long ncell = (long)dims[0] * dims[1] * dims[2];
    double M = 0.0, J[3] = {0.0, 0.0, 0.0};
    for (long c = 0; c < ncell; ++c) {
        if (solid[c]) continue;
        for (int i = 0; i < Q; ++i) {
            double f = A[i * ncell + c];
            M += f;
            for (int a = 0; a < 3; ++a) J[a] += CV[i][a] * f;
        }
    }
    out[0] = M;
    out[1] = J[0];
    out[2] = J[1];
    out[3] = J[2];
}

/* Density and physical velocity u = (j + rho g / 2) / rho of every fluid
 * cell: out[0][c] = rho, out[1..3][c] = u. Solid cells get zeros. */
void ora_macroscopic(const double *A, const uint8_t *solid, const int dims[3], const double g[3], double *out)
{
    init_tables();
    const long ncell = (long)dims[0] * dims[1] * dims[2];
    for (long c = 0; c < ncell; ++c) {
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        if (!solid[c]) {
            for (int i = 0; i < Q; ++i) {
                double f = A[i * ncell + c];
                rho += f;
                for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * f;
            }
        }
        out[c] = rho;
        for (int a = 0; a < 3; ++a) out[(a + 1) * ncell + c] = solid[c] ? 0.0 : (j[a] + 0.5 * rho * g[a]) / rho;
    }
}

/* f = f^eq(rho, u) on every fluid cell; rho_u[0][c] = rho, rho_u[1..3][c] = u. */
void ora_init_equilibrium(const double *rho_u, const uint8_t *solid, const int dims[3], double *A)
{
    init_tables();
    const long ncell = (long)dims[0] * dims[1] * dims[2];
    for (long c = 0; c < ncell; ++c) {
        double feq[Q] = {0};
        if (!solid[c]) {
            double u[3] = {rho_u[ncell + c], rho_u[2 * ncell + c], rho_u[3 * ncell + c]};
            ora_equilibrium(rho_u[c], u, feq);
        }
        for (int i = 0; i < Q; ++i) A[i * ncell + c] = feq[i];
    }
}

/* Index array of indirect addressing.  Fluid ids number the fluid cells in
 * a traversal order: bricks of bx*by*bz cells taken in lexicographic brick
 * order, the cells of a brick in lexicographic order, cells outside the box
 * skipped (the paper benchmarks several such setups of the sparse
 * representation, Sec. 10).  A brick equal to the whole box (or 0 in any
 * dimension) is the plain lexicographic order, x fastest.
 * cellmap[c] = fluid id or -1.  idx (optional, 18 rows of idx_pitch):
 * idx[k][n] = id of the cell at x_n + c_{k+1}, -1 if solid or outside a
 * non-periodic axis, -m for a boundary cell of mask value 2 <= m <= 5.  Returns
 * the number of fluid nodes. */
long ora_build_idx_brick(const uint8_t *solid, const int dims[3], const int periodic[3], const int brick[3],
                         int32_t *cellmap, int32_t *idx, long idx_pitch)
{
    init_tables();
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const long ncell = (long)nx * ny * nz;
    int b[3];
    for (int a = 0; a < 3; ++a) b[a] = (brick && brick[a] > 0) ? brick[a] : dims[a];
    long nf = 0;
    for (long c = 0; c < ncell; ++c) cellmap[c] = -1;
    for (int Bz = 0; Bz < nz; Bz += b[2])
        for (int By = 0; By < ny; By += b[1])
            for (int Bx = 0; Bx < nx; Bx += b[0])
                for (int z = Bz; z < Bz + b[2] && z < nz; ++z)
                    for (int y = By; y < By + b[1] && y < ny; ++y)
                        for (int x = Bx; x < Bx + b[0] && x < nx; ++x) {
                            long c = x + (long)nx * (y + (long)ny * z);
                            if (!solid[c]) cellmap[c] = (int32_t)nf++;
                        }
    if (!idx) return nf;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = x + (long)nx * (y + (long)ny * z);
                if (solid[c]) continue;
                long n = cellmap[c];
                for (int k = 0; k < Q - 1; ++k) {
                    int i = k + 1;
                    int p[3] = {x + CV[i][0], y + CV[i][1], z + CV[i][2]};
                    int out = 0;
                    for (int a = 0; a < 3; ++a) {
                        if (p[a] < 0 || p[a] >= dims[a]) {
                            if (!periodic[a]) out = 1;
                            else p[a] = (p[a] + dims[a]) % dims[a];
                        }
                    }
                    int32_t v = -1;
                    if (!out) {
                        long cc = p[0] + (long)nx * (p[1] + (long)ny * p[2]);
                        const int mv = solid[cc];
                        v = (mv >= 2 && mv <= 5) ? -mv : (mv ? -1 : cellmap[cc]);
                    }
                    idx[k * idx_pitch + n] = v;
                }
            }
    return nf;
}

/* Lexicographic order (x fastest): the whole box is one brick. */
long ora_build_idx(const uint8_t *solid, const int dims[3], const int periodic[3], int32_t *cellmap,
                   int32_t *idx, long idx_pitch)
{
    return ora_build_idx_brick(solid, dims, periodic, 0, cellmap, idx, idx_pitch);
}

int ora_num_threads(int nthreads)
{
    return resolve_threads(nthreads);
}
