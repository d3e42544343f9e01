/*
 * Plain FP64 CPU reference ("oracle") of the two-component lattice Boltzmann
 * time step on the D3Q19 lattice, the lattice of the paper's 3-D runs (Sec. 2),
 * for the sinusoidal tube of Sec. 3.4 and periodic boxes.
 *
 * TEST INFRASTRUCTURE.  Only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark load this file.  It shares no code, header, table or helper with
 * the HIP library.  Same model and readings as the D2Q9 oracle (lbm_oracle.c):
 * Eq. 7 third-order equilibrium, Eq. 6 regularization with the species' own
 * non-equilibrium momentum flux, Eq. 8 interaction with wall potentials, the
 * force folded into the equilibrium velocity (Eq. 9), Eqs. 4-5 mixed relaxation,
 * half-way bounce-back at solid links.  Deliberately slow and literal; built
 * with -O2 -ffp-contract=off.
 *
 * Lattice: D3Q19, T0 = 1/3.
 *   i = 0           rest                          w = 1/3
 *   i = 1 .. 6      (+-1,0,0), (0,+-1,0), (0,0,+-1)  w = 1/18
 *   i = 7 .. 18     the 12 face diagonals            w = 1/36
 * (the order is fixed by the tables below; opp(i) is the reversed direction).
 *
 * Arrays (row-major, x fastest):
 *   f    [2][19][nz][ny][nx]   populations after streaming (state at time t)
 *   rho  [2][nz][ny][nx]
 *   mask [nz][ny][nx]          1 = fluid
 * x is always periodic; y and z are periodic when periodic_yz != 0, otherwise a
 * node outside the box counts as solid.
 *
 * Walls: half-way bounce-back at solid links (default), or, with wall_interp,
 * the analytic sinusoidal tube wall (y - yc)^2 + (z - zc)^2 = r(x)^2,
 * r(x) = r0 + a cos(2 pi x / lambda), at its sub-lattice position by linear
 * interpolated bounce-back with the mass returned through the rest population
 * (orc3_step_interp), as the D2Q9 oracle does for its channel walls.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q3 19

static const int CX3[Q3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY3[Q3] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ3[Q3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
static const double T03 = 1.0 / 3.0;

static double weight3(int i)
{
    const int n = abs(CX3[i]) + abs(CY3[i]) + abs(CZ3[i]);
    return n == 0 ? 1.0 / 3.0 : (n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

static int opposite3(int i)
{
    for (int j = 0; j < Q3; ++j)
        if (CX3[j] == -CX3[i] && CY3[j] == -CY3[i] && CZ3[j] == -CZ3[i])
            return j;
    return -1;
}

typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic_yz;
    double tau[2];
    double G;
    double rho_s[2];
    double g[3];
    /* Interpolated tube walls (wall_interp != 0): axis (wall_yc, wall_zc),
     * radius wall_r0 + wall_a cos(2 pi x / wall_lam). */
    int32_t wall_interp;
    int32_t reserved;
    double wall_yc, wall_zc, wall_r0, wall_a, wall_lam;
} orc3_params;

void orc3_lattice(int *cx, int *cy, int *cz, double *w, int *opp)
{
    for (int i = 0; i < Q3; ++i) {
        cx[i] = CX3[i];
        cy[i] = CY3[i];
        cz[i] = CZ3[i];
        w[i] = weight3(i);
        opp[i] = opposite3(i);
    }
}

static int wrap3(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

static int fluid3(const orc3_params *p, const uint8_t *mask, int x, int y, int z)
{
    x = wrap3(x, p->nx);
    if (p->periodic_yz) {
        y = wrap3(y, p->ny);
        z = wrap3(z, p->nz);
    } else if (y < 0 || y >= p->ny || z < 0 || z >= p->nz) {
        return 0;
    }
    return mask[((size_t)z * p->ny + y) * p->nx + x] != 0;
}

static size_t index3(const orc3_params *p, int x, int y, int z)
{
    return ((size_t)wrap3(z, p->nz) * p->ny + wrap3(y, p->ny)) * p->nx + wrap3(x, p->nx);
}

/* Eq. 7 on D3Q19. */
void orc3_equilibrium(double rho, double ux, double uy, double uz, double *feq)
{
    const double usq = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < Q3; ++i) {
        const double cu = CX3[i] * ux + CY3[i] * uy + CZ3[i] * uz;
        const double bracket = 1.0
                             + cu / T03
                             + (cu * cu) / (2.0 * T03 * T03)
                             - usq / (2.0 * T03)
                             + (cu * cu * cu) / (6.0 * T03 * T03 * T03)
                             - cu * usq / (2.0 * T03 * T03);
        feq[i] = rho * weight3(i) * bracket;
    }
}

/* Eq. 6: f'_i = w_i / (2 T0^2) H_i : Pi^neq, H_i = c_i c_i - T0 I. */
void orc3_regularize(const double *f, const double *feq, double *fneq)
{
    double P[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int i = 0; i < Q3; ++i) {
        const int c[3] = {CX3[i], CY3[i], CZ3[i]};
        const double d = f[i] - feq[i];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                P[a][b] += c[a] * c[b] * d;
    }
    for (int i = 0; i < Q3; ++i) {
        const int c[3] = {CX3[i], CY3[i], CZ3[i]};
        double contraction = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                contraction += (c[a] * c[b] - (a == b ? T03 : 0.0)) * P[a][b];
        fneq[i] = weight3(i) / (2.0 * T03 * T03) * contraction;
    }
}

void orc3_densities(const orc3_params *p, const uint8_t *mask, const double *f, double *rho)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    for (int s = 0; s < 2; ++s)
        for (size_t k = 0; k < n; ++k) {
            double r = 0.0;
            if (mask[k])
                for (int i = 0; i < Q3; ++i)
                    r += f[((size_t)s * Q3 + i) * n + k];
            rho[(size_t)s * n + k] = r;
        }
}

/* Eq. 8 with wall potentials: S^beta = sum_i w_i c_i rho~^beta(x + c_i). */
static void interaction3(const orc3_params *p, const uint8_t *mask, const double *rho, int beta,
                         int x, int y, int z, double *S)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    S[0] = S[1] = S[2] = 0.0;
    for (int i = 1; i < Q3; ++i) {
        const int xn = x + CX3[i], yn = y + CY3[i], zn = z + CZ3[i];
        const double rb = fluid3(p, mask, xn, yn, zn)
                              ? rho[(size_t)beta * n + index3(p, xn, yn, zn)]
                              : p->rho_s[beta];
        S[0] += weight3(i) * CX3[i] * rb;
        S[1] += weight3(i) * CY3[i] * rb;
        S[2] += weight3(i) * CZ3[i] * rb;
    }
}

static double tau_mix3(const orc3_params *p, double ro, double rw)
{
    const double nu_o = T03 * (p->tau[0] - 0.5), nu_w = T03 * (p->tau[1] - 0.5);
    return (ro * nu_o + rw * nu_w) / (ro + rw) / T03 + 0.5;
}

typedef struct {
    double rho[2], j[2][3], u[3], F[2][3];
} node3;

static void gather3(const orc3_params *p, const uint8_t *mask, const double *f,
                    const double *rho_field, int x, int y, int z, node3 *st)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const size_t k = index3(p, x, y, z);
    for (int s = 0; s < 2; ++s) {
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < Q3; ++i) {
            const double v = f[((size_t)s * Q3 + i) * n + k];
            r += v;
            j[0] += CX3[i] * v;
            j[1] += CY3[i] * v;
            j[2] += CZ3[i] * v;
        }
        st->rho[s] = r;
        for (int a = 0; a < 3; ++a)
            st->j[s][a] = j[a];
    }
    const double rt = st->rho[0] + st->rho[1];
    for (int a = 0; a < 3; ++a)
        st->u[a] = (st->j[0][a] + st->j[1][a]) / rt;
    for (int s = 0; s < 2; ++s) {
        double S[3];
        interaction3(p, mask, rho_field, 1 - s, x, y, z, S);
        for (int a = 0; a < 3; ++a)
            st->F[s][a] = p->G * st->rho[s] * S[a] + st->rho[s] * p->g[a];
    }
}

static int orc3_step_interp(const orc3_params *p, const uint8_t *mask, const double *f_in,
                            double *f_out, double *rho_work);

/* One step, f_in (time t) -> f_out (time t + 1).  Returns the number of fluid
 * nodes whose densities were not finite and positive. */

int orc3_step(const orc3_params *p, const uint8_t *mask, const double *f_in, double *f_out,
              double *rho_work)
{
    if (p->wall_interp)
        return orc3_step_interp(p, mask, f_in, f_out, rho_work);
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t n = (size_t)nx * ny * nz;
    int bad = 0;
    orc3_densities(p, mask, f_in, rho_work);
    memset(f_out, 0, sizeof(double) * 2 * Q3 * n);
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t k = index3(p, x, y, z);
                if (!mask[k])
                    continue;
                node3 st;
                gather3(p, mask, f_in, rho_work, x, y, z, &st);
                if (!(st.rho[0] > 0.0) || !(st.rho[1] > 0.0) || !isfinite(st.rho[0] + st.rho[1]))
                    ++bad;
                const double taum = tau_mix3(p, st.rho[0], st.rho[1]);
                for (int s = 0; s < 2; ++s) {
                    double fl[Q3], feq_own[Q3], feq_shift[Q3], fneq[Q3];
                    for (int i = 0; i < Q3; ++i)
                        fl[i] = f_in[((size_t)s * Q3 + i) * n + k];
                    orc3_equilibrium(st.rho[s], st.u[0] + st.F[s][0] / st.rho[s],
                                     st.u[1] + st.F[s][1] / st.rho[s],
                                     st.u[2] + st.F[s][2] / st.rho[s], feq_shift);
                    orc3_equilibrium(st.rho[s], st.j[s][0] / st.rho[s], st.j[s][1] / st.rho[s],
                                     st.j[s][2] / st.rho[s], feq_own);
                    orc3_regularize(fl, feq_own, fneq);
                    for (int i = 0; i < Q3; ++i) {
                        const double post = feq_shift[i] + (1.0 - 1.0 / taum) * fneq[i];
                        const int xn = x + CX3[i], yn = y + CY3[i], zn = z + CZ3[i];
                        if (fluid3(p, mask, xn, yn, zn))
                            f_out[((size_t)s * Q3 + i) * n + index3(p, xn, yn, zn)] = post;
                        else
                            f_out[((size_t)s * Q3 + opposite3(i)) * n + k] = post;
                    }
                }
            }
    return bad;
}

/* Inside the analytic tube (the voxelisation's own expression, at any point). */
static int tube_inside(const orc3_params *p, double X, double Y, double Z)
{
    const double r = p->wall_r0 + p->wall_a * cos(6.283185307179586476925286766559 * X /
                                                 p->wall_lam);
    const double dy = Y - p->wall_yc, dz = Z - p->wall_zc;
    return dy * dy + dz * dz < r * r;
}

/* Fraction q in (0, 1] of the link from fluid node (x, y, z) along c_i at
 * which it leaves the tube: 60 halvings of the link, keeping the first point
 * found outside. */
double orc3_wall_fraction(const orc3_params *p, int x, int y, int z, int i)
{
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
        const double t = 0.5 * (lo + hi);
        if (tube_inside(p, x + t * CX3[i], y + t * CY3[i], z + t * CZ3[i]))
            lo = t;
        else
            hi = t;
    }
    return hi;
}

/* Collision of one fluid node (the same arithmetic as orc3_step), returning
 * the post-collision populations of both species. */
static int collide3(const orc3_params *p, const uint8_t *mask, const double *f_in,
                    const double *rho_work, int x, int y, int z, double post[2][Q3])
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const size_t k = index3(p, x, y, z);
    node3 st;
    gather3(p, mask, f_in, rho_work, x, y, z, &st);
    const int bad = (!(st.rho[0] > 0.0) || !(st.rho[1] > 0.0) ||
                     !isfinite(st.rho[0] + st.rho[1])) ? 1 : 0;
    const double taum = tau_mix3(p, st.rho[0], st.rho[1]);
    for (int s = 0; s < 2; ++s) {
        double fl[Q3], feq_own[Q3], feq_shift[Q3], fneq[Q3];
        for (int i = 0; i < Q3; ++i)
            fl[i] = f_in[((size_t)s * Q3 + i) * n + k];
        orc3_equilibrium(st.rho[s], st.u[0] + st.F[s][0] / st.rho[s],
                         st.u[1] + st.F[s][1] / st.rho[s], st.u[2] + st.F[s][2] / st.rho[s],
                         feq_shift);
        orc3_equilibrium(st.rho[s], st.j[s][0] / st.rho[s], st.j[s][1] / st.rho[s],
                         st.j[s][2] / st.rho[s], feq_own);
        orc3_regularize(fl, feq_own, fneq);
        for (int i = 0; i < Q3; ++i)
            post[s][i] = feq_shift[i] + (1.0 - 1.0 / taum) * fneq[i];
    }
    return bad;
}

/* One step with interpolated tube walls: collide every node, then stream; a
 * population leaving fluid node x along c_i towards a wall met at the fraction
 * q of the link returns as f_opp(i)(x) by the linear interpolated bounce-back
 * of Bouzidi, Firdaouss and Lallemand (2001):
 *   q <  1/2: 2q f*_i(x) + (1 - 2q) f*_i(x - c_i)   (f*_i(x) if x - c_i is solid)
 *   q >= 1/2: f*_i(x) / (2q) + (1 - 1/(2q)) f*_opp(i)(x)
 * and what the blends add beyond half-way bounce-back is taken from the node's
 * rest population, so each species keeps its mass. */
static int orc3_step_interp(const orc3_params *p, const uint8_t *mask, const double *f_in,
                            double *f_out, double *rho_work)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t n = (size_t)nx * ny * nz;
    int bad = 0;
    orc3_densities(p, mask, f_in, rho_work);
    double *post = (double *)calloc(2 * Q3 * n, sizeof(double));
    if (!post)
        return -1;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t k = index3(p, x, y, z);
                if (!mask[k])
                    continue;
                double fp[2][Q3];
                bad += collide3(p, mask, f_in, rho_work, x, y, z, fp);
                for (int s = 0; s < 2; ++s)
                    for (int i = 0; i < Q3; ++i)
                        post[((size_t)s * Q3 + i) * n + k] = fp[s][i];
            }
    memset(f_out, 0, sizeof(double) * 2 * Q3 * n);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t k = index3(p, x, y, z);
                if (!mask[k])
                    continue;
                for (int s = 0; s < 2; ++s) {
                    double dm = 0.0;
                    for (int i = 0; i < Q3; ++i) {
                        const double v = post[((size_t)s * Q3 + i) * n + k];
                        const int xn = x + CX3[i], yn = y + CY3[i], zn = z + CZ3[i];
                        if (fluid3(p, mask, xn, yn, zn)) {
                            f_out[((size_t)s * Q3 + i) * n + index3(p, xn, yn, zn)] = v;
                            continue;
                        }
                        const double q = orc3_wall_fraction(p, x, y, z, i);
                        double back;
                        if (q < 0.5) {
                            const int xb = x - CX3[i], yb = y - CY3[i], zb = z - CZ3[i];
                            back = fluid3(p, mask, xb, yb, zb)
                                       ? 2.0 * q * v + (1.0 - 2.0 * q) *
                                             post[((size_t)s * Q3 + i) * n + index3(p, xb, yb, zb)]
                                       : v;
                        } else {
                            back = v / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) *
                                                       post[((size_t)s * Q3 + opposite3(i)) * n + k];
                        }
                        f_out[((size_t)s * Q3 + opposite3(i)) * n + k] = back;
                        dm += back - v;
                    }
                    f_out[((size_t)s * Q3 + 0) * n + k] -= dm;
                }
            }
    free(post);
    return bad;
}

int64_t orc3_run(const orc3_params *p, const uint8_t *mask, double *f, double *work,
                 int64_t nsteps)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    double *other = work, *rho = work + 2 * Q3 * n;
    for (int64_t t = 0; t < nsteps; ++t) {
        const int bad = orc3_step(p, mask, f, other, rho);
        memcpy(f, other, sizeof(double) * 2 * Q3 * n);
        if (bad)
            return t;
    }
    return -1;
}

void orc3_init(const orc3_params *p, const uint8_t *mask, const double *rho0, double *f)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    memset(f, 0, sizeof(double) * 2 * Q3 * n);
    for (int s = 0; s < 2; ++s)
        for (size_t k = 0; k < n; ++k) {
            if (!mask[k])
                continue;
            double feq[Q3];
            orc3_equilibrium(rho0[(size_t)s * n + k], 0.0, 0.0, 0.0, feq);
            for (int i = 0; i < Q3; ++i)
                f[((size_t)s * Q3 + i) * n + k] = feq[i];
        }
}

/* rho_out [2][n], u_out [3][n] (physical mixture velocity u_mix + (F^o + F^w)
 * / (2 rho)), p_out [n] (T0 rho - G T0 rho^o rho^w), mon [8] (sum rho^o,
 * sum rho^w, physical momentum x, y, sum rho^o u_x, sum rho^o cos(2 pi x/nx),
 * sum rho^o sin(2 pi x/nx), bad nodes).  Outputs may be NULL. */
void orc3_moments(const orc3_params *p, const uint8_t *mask, const double *f, double *rho_work,
                  double *rho_out, double *u_out, double *p_out, double *mon)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const double two_pi = 6.283185307179586476925286766559;
    double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    orc3_densities(p, mask, f, rho_work);
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const size_t k = index3(p, x, y, z);
                double r0 = 0, r1 = 0, u[3] = {0, 0, 0}, pr = 0;
                if (mask[k]) {
                    node3 st;
                    gather3(p, mask, f, rho_work, x, y, z, &st);
                    const double rt = st.rho[0] + st.rho[1];
                    double P[3];
                    for (int a = 0; a < 3; ++a) {
                        P[a] = st.j[0][a] + st.j[1][a] + 0.5 * (st.F[0][a] + st.F[1][a]);
                        u[a] = P[a] / rt;
                    }
                    r0 = st.rho[0];
                    r1 = st.rho[1];
                    pr = T03 * rt - p->G * T03 * r0 * r1;
                    m[0] += r0;
                    m[1] += r1;
                    m[2] += P[0];
                    m[3] += P[1];
                    m[4] += r0 * u[0];
                    m[5] += r0 * cos(two_pi * x / p->nx);
                    m[6] += r0 * sin(two_pi * x / p->nx);
                    if (!(r0 > 0.0) || !(r1 > 0.0) || !isfinite(r0 + r1 + u[0] + u[1] + u[2]))
                        m[7] += 1.0;
                }
                if (rho_out) {
                    rho_out[k] = r0;
                    rho_out[n + k] = r1;
                }
                if (u_out)
                    for (int a = 0; a < 3; ++a)
                        u_out[(size_t)a * n + k] = u[a];
                if (p_out)
                    p_out[k] = pr;
            }
    if (mon)
        for (int j = 0; j < 8; ++j)
            mon[j] = m[j];
}
