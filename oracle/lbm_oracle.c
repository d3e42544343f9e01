/*
 * Plain FP64 CPU reference ("oracle") of the two-component lattice Boltzmann
 * time step of Otomo et al., "Simulation of residual oil displacement in a
 * sinusoidal channel with the lattice Boltzmann method" (arXiv 1601.00918).
 *
 * TEST INFRASTRUCTURE.  Only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark load this file.  It shares no code, header, table or helper with
 * the HIP library; the two are compared element by element.
 *
 * The code is deliberately slow and literal: every node recomputes everything it
 * needs, the equilibria are evaluated direction by direction, and the non-
 * equilibrium momentum flux is taken as the second moment of f - f^eq exactly as
 * it is defined.  Built with -O2 -ffp-contract=off (no FMA contraction, no fast
 * math), so every result is IEEE binary64 round-to-nearest-even.
 *
 * Lattice: D2Q9 (the paper's 2-D cases; its 3-D runs use D3Q19, Sec. 2).
 *   i   : 0      1      2      3       4       5      6       7        8
 *   c_i : (0,0)  (1,0)  (0,1)  (-1,0)  (0,-1)  (1,1)  (-1,1)  (-1,-1)  (1,-1)
 *   w_i : 4/9    1/9    1/9    1/9     1/9     1/36   1/36    1/36     1/36
 *   lattice temperature T0 = 1/3 (Sec. 2, after Eq. 5).
 *
 * Species index s: 0 = oil ("o", species A), 1 = water ("w", species B).
 *
 * Array layout (all row-major, x fastest):
 *   f    [2][9][ny][nx]   populations after streaming, i.e. the state at time t
 *   rho  [2][ny][nx]
 *   mask [ny][nx]         1 = fluid node, 0 = solid node
 *
 * Geometry: x is always periodic.  y is periodic when periodic_y != 0; otherwise
 * a node outside 0 <= y < ny counts as solid.
 *
 * Regularization: second-order Hermite projection of the non-equilibrium part
 * (Eq. 6, the default), or with reg_order = 3 also its third-order Hermite
 * projection (orc_regularize3), the higher-order variant of the cited schemes.
 *
 * Walls: half-way bounce-back at solid links (default), or, with wall_interp,
 * the analytic channel walls at their sub-lattice positions by linear
 * interpolated bounce-back (orc_step_interp), which places the wall where the
 * geometry puts it at the price of exact mass conservation.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

static const int CXI[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CYI[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPPOSITE[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WEIGHT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                                 1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                                 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double T0 = 1.0 / 3.0;

typedef struct {
    int32_t nx, ny;
    int32_t periodic_y;
    int32_t reg_order; /* Hermite order of the regularization: 2 (0 means 2) or 3 */
    double tau[2];   /* single-species relaxation times tau^o, tau^w */
    double G;        /* interaction strength of Eq. 8 (repulsion: G < 0) */
    double rho_s[2]; /* wall potentials rho_s^o, rho_s^w (Sec. 2, last paragraph) */
    double g[2];     /* homogeneous body acceleration (Sec. 3.4) */
    /* Interpolated walls (wall_interp != 0): the channel walls
     * y = wall_yc +- (wall_h0 + wall_a cos(2 pi x / wall_lam)) placed at their
     * sub-lattice positions by linear interpolated bounce-back. */
    int32_t wall_interp;
    int32_t reserved2;
    double wall_yc, wall_h0, wall_a, wall_lam;
} orc_params;

/* ---- lattice constants, exported so tests can check them ------------------ */
/* Threads of the OpenMP row loops (timing only: results do not depend on it). */
void orc_set_threads(int n)
{
    if (n > 0)
        omp_set_num_threads(n);
}

int orc_get_threads(void) { return omp_get_max_threads(); }

void orc_lattice(int *cx, int *cy, double *w, int *opp)
{
    for (int i = 0; i < Q; ++i) {
        cx[i] = CXI[i];
        cy[i] = CYI[i];
        w[i] = WEIGHT[i];
        opp[i] = OPPOSITE[i];
    }
}

/* ---- geometry ------------------------------------------------------------- */
static int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Is (x, y) a fluid node?  x wraps; y wraps only for periodic_y. */
static int node_is_fluid(const orc_params *p, const uint8_t *mask, int x, int y)
{
    x = wrap(x, p->nx);
    if (p->periodic_y)
        y = wrap(y, p->ny);
    else if (y < 0 || y >= p->ny)
        return 0;
    return mask[(size_t)y * p->nx + x] != 0;
}

static size_t node_index(const orc_params *p, int x, int y)
{
    x = wrap(x, p->nx);
    y = wrap(y, p->ny);
    return (size_t)y * p->nx + x;
}

/* ---- Eq. 7: third-order equilibrium --------------------------------------- */
void orc_equilibrium(double rho, double ux, double uy, double *feq)
{
    const double usq = ux * ux + uy * uy;
    for (int i = 0; i < Q; ++i) {
        const double cu = CXI[i] * ux + CYI[i] * uy;
        const double bracket = 1.0
                             + cu / T0
                             + (cu * cu) / (2.0 * T0 * T0)
                             - usq / (2.0 * T0)
                             + (cu * cu * cu) / (6.0 * T0 * T0 * T0)
                             - cu * usq / (2.0 * T0 * T0);
        feq[i] = rho * WEIGHT[i] * bracket;
    }
}

/* ---- Eq. 6: regularized non-equilibrium part -------------------------------
 * Pi^neq = sum_i c_i c_i (f_i - feq_i) is the non-equilibrium momentum flux; the
 * regularization keeps only its projection on the second-order Hermite
 * polynomials H_i = c_i c_i - T0 I:
 *   f'_i = w_i / (2 T0^2) * H_i : Pi^neq.                                      */
void orc_regularize(const double *f, const double *feq, double *fneq, double *pi_neq)
{
    double pxx = 0.0, pxy = 0.0, pyy = 0.0;
    for (int i = 0; i < Q; ++i) {
        const double d = f[i] - feq[i];
        pxx += CXI[i] * CXI[i] * d;
        pxy += CXI[i] * CYI[i] * d;
        pyy += CYI[i] * CYI[i] * d;
    }
    for (int i = 0; i < Q; ++i) {
        const double hxx = CXI[i] * CXI[i] - T0;
        const double hxy = CXI[i] * CYI[i];
        const double hyy = CYI[i] * CYI[i] - T0;
        const double contraction = hxx * pxx + 2.0 * hxy * pxy + hyy * pyy;
        fneq[i] = WEIGHT[i] / (2.0 * T0 * T0) * contraction;
    }
    if (pi_neq) {
        pi_neq[0] = pxx;
        pi_neq[1] = pxy;
        pi_neq[2] = pyy;
    }
}

/* ---- Eq. 6 with the third-order Hermite terms (regularization of the cited
 * higher-order schemes): besides the second-order projection above, f - feq is
 * projected on the third-order Hermite polynomials
 *   H3_i,abc = c_a c_b c_c - T0 (c_a d_bc + c_b d_ac + c_c d_ab),
 *   a3_abc = sum_i H3_i,abc (f_i - feq_i),
 *   f'_i += w_i / (6 T0^3) * sum_abc H3_i,abc a3_abc   (all 8 index triples).
 * a3_out (may be NULL) receives a3 as [a][b][c], 8 values.                   */
void orc_regularize3(const double *f, const double *feq, double *fneq, double *a3_out)
{
    orc_regularize(f, feq, fneq, NULL);
    double a3[2][2][2];
    int c[Q][2];
    for (int i = 0; i < Q; ++i) {
        c[i][0] = CXI[i];
        c[i][1] = CYI[i];
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int g = 0; g < 2; ++g) {
                double sum = 0.0;
                for (int i = 0; i < Q; ++i) {
                    const double h = c[i][a] * c[i][b] * c[i][g]
                                   - T0 * (c[i][a] * (b == g) + c[i][b] * (a == g) + c[i][g] * (a == b));
                    sum += h * (f[i] - feq[i]);
                }
                a3[a][b][g] = sum;
            }
    for (int i = 0; i < Q; ++i) {
        double contraction = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int g = 0; g < 2; ++g) {
                    const double h = c[i][a] * c[i][b] * c[i][g]
                                   - T0 * (c[i][a] * (b == g) + c[i][b] * (a == g) + c[i][g] * (a == b));
                    contraction += h * a3[a][b][g];
                }
        fneq[i] += WEIGHT[i] / (6.0 * T0 * T0 * T0) * contraction;
    }
    if (a3_out)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int g = 0; g < 2; ++g)
                    a3_out[(a * 2 + b) * 2 + g] = a3[a][b][g];
}

/* ---- per-node densities of both species (solid nodes: 0) ------------------ */
void orc_densities(const orc_params *p, const uint8_t *mask, const double *f, double *rho)
{
    const size_t n = (size_t)p->nx * p->ny;
    for (int s = 0; s < 2; ++s)
        for (size_t k = 0; k < n; ++k) {
            double r = 0.0;
            if (mask[k])
                for (int i = 0; i < Q; ++i)
                    r += f[((size_t)s * Q + i) * n + k];
            rho[(size_t)s * n + k] = r;
        }
}

/* ---- Eq. 8 with wall potentials --------------------------------------------
 * S^beta(x) = sum_i w_i c_i rho~^beta(x + c_i), where rho~^beta is the density of
 * species beta at a fluid neighbour and the wall potential rho_s^beta at a solid
 * one.  The force on species alpha is then F^{alpha beta} = G rho^alpha S^beta. */
void orc_interaction_sum(const orc_params *p, const uint8_t *mask, const double *rho,
                         int beta, int x, int y, double *sx, double *sy)
{
    const size_t n = (size_t)p->nx * p->ny;
    double ax = 0.0, ay = 0.0;
    for (int i = 1; i < Q; ++i) {
        const int xn = x + CXI[i], yn = y + CYI[i];
        double rb;
        if (node_is_fluid(p, mask, xn, yn))
            rb = rho[(size_t)beta * n + node_index(p, xn, yn)];
        else
            rb = p->rho_s[beta];
        ax += WEIGHT[i] * CXI[i] * rb;
        ay += WEIGHT[i] * CYI[i] * rb;
    }
    *sx = ax;
    *sy = ay;
}

/* ---- Eqs. 4-5: mixed relaxation time ---------------------------------------- */
double orc_tau_mix(const orc_params *p, double rho_o, double rho_w)
{
    const double nu_o = T0 * (p->tau[0] - 0.5);
    const double nu_w = T0 * (p->tau[1] - 0.5);
    const double nu_mix = (rho_o * nu_o + rho_w * nu_w) / (rho_o + rho_w);
    return nu_mix / T0 + 0.5;
}

/* Node state shared by the step and the moments: densities, momenta, mixture
 * velocity (Eq. 10), total force per species (Eq. 8 + body force). */
typedef struct {
    double rho[2], jx[2], jy[2];
    double ux, uy;          /* u_mix, Eq. 10 */
    double fx[2], fy[2];    /* F^alpha = G rho^alpha S^beta + rho^alpha g */
} node_state;

static void gather_node(const orc_params *p, const uint8_t *mask, const double *f,
                        const double *rho_field, int x, int y, node_state *st)
{
    const size_t n = (size_t)p->nx * p->ny;
    const size_t k = (size_t)y * p->nx + x;
    for (int s = 0; s < 2; ++s) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < Q; ++i) {
            const double v = f[((size_t)s * Q + i) * n + k];
            r += v;
            jx += CXI[i] * v;
            jy += CYI[i] * v;
        }
        st->rho[s] = r;
        st->jx[s] = jx;
        st->jy[s] = jy;
    }
    const double rho_tot = st->rho[0] + st->rho[1];
    st->ux = (st->jx[0] + st->jx[1]) / rho_tot;
    st->uy = (st->jy[0] + st->jy[1]) / rho_tot;
    for (int s = 0; s < 2; ++s) {
        const int beta = 1 - s;
        double sx, sy;
        orc_interaction_sum(p, mask, rho_field, beta, x, y, &sx, &sy);
        st->fx[s] = p->G * st->rho[s] * sx + st->rho[s] * p->g[0];
        st->fy[s] = p->G * st->rho[s] * sy + st->rho[s] * p->g[1];
    }
}

/* ---- one time step: collide (Eqs. 3-10) then stream (Eq. 1) ----------------
 * f_in: state at time t; f_out: state at time t+1 (fully overwritten; solid
 * nodes are set to 0).  rho_work: [2][ny][nx] scratch.  Returns the number of
 * fluid nodes whose densities were not finite and positive (0 on success). */
/* Fraction q in (0, 1] of the link from fluid node (x, y) along c_i at which
 * it crosses the analytic channel wall: in closed form for flat walls,
 * otherwise by bisection on the segment, returning the upper end of the final
 * interval. */
double orc_wall_fraction(const orc_params *p, int x, int y, int i)
{
    const double two_pi = 6.283185307179586476925286766559;
    if (p->wall_a == 0.0) /* flat walls: links meet them along y only */
        return (p->wall_h0 - fabs(y - p->wall_yc)) / fabs((double)CYI[i]);
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
        const double t = 0.5 * (lo + hi);
        const double X = x + t * CXI[i], Y = y + t * CYI[i];
        const double h = p->wall_h0 + p->wall_a * cos(two_pi * X / p->wall_lam);
        if (fabs(Y - p->wall_yc) < h)
            lo = t;
        else
            hi = t;
    }
    return hi; /* first point found outside: a wall exactly half-way gives 1/2 */
}

/* Post-collision populations of both species at fluid node (x, y), Eq. 3. */
static int collide_node(const orc_params *p, const uint8_t *mask, const double *f_in,
                        const double *rho_work, int x, int y, double fpost[2][Q])
{
    const size_t n = (size_t)p->nx * p->ny;
    const size_t k = (size_t)y * p->nx + x;
    node_state st;
    gather_node(p, mask, f_in, rho_work, x, y, &st);
    const int bad = (!(st.rho[0] > 0.0) || !(st.rho[1] > 0.0) || !isfinite(st.rho[0] + st.rho[1]));
    const double tau_mix = orc_tau_mix(p, st.rho[0], st.rho[1]);
    for (int s = 0; s < 2; ++s) {
        double fl[Q], feq_own[Q], feq_shift[Q], fneq[Q];
        for (int i = 0; i < Q; ++i)
            fl[i] = f_in[((size_t)s * Q + i) * n + k];
        orc_equilibrium(st.rho[s], st.ux + st.fx[s] / st.rho[s], st.uy + st.fy[s] / st.rho[s],
                        feq_shift);
        orc_equilibrium(st.rho[s], st.jx[s] / st.rho[s], st.jy[s] / st.rho[s], feq_own);
        if (p->reg_order == 3)
            orc_regularize3(fl, feq_own, fneq, NULL);
        else
            orc_regularize(fl, feq_own, fneq, NULL);
        for (int i = 0; i < Q; ++i)
            fpost[s][i] = feq_shift[i] + (1.0 - 1.0 / tau_mix) * fneq[i];
    }
    return bad;
}

/* One step with interpolated walls: collide every node, then stream; a
 * population f*_i(x) leaving towards a wall that the link crosses at fraction
 * q returns as f_opp(i)(x) by the linear interpolated bounce-back of Bouzidi,
 * Firdaouss and Lallemand (2001):
 *   q <  1/2:  2q f*_i(x) + (1 - 2q) f*_i(x - c_i)     (x - c_i fluid; else f*_i(x))
 *   q >= 1/2:  f*_i(x) / (2q) + (1 - 1/(2q)) f*_opp(i)(x)
 * and the node's rest population gives back what the returned populations
 * carry beyond f*_i(x), so each species' mass is kept exactly (with the wall
 * potentials' force in the post-collision populations the plain scheme gains
 * mass at every wall link).  q = 1/2 is the half-way bounce-back of orc_step. */
static int orc_step_interp(const orc_params *p, const uint8_t *mask, const double *f_in,
                           double *f_out, double *rho_work)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    int bad = 0;
    orc_densities(p, mask, f_in, rho_work);
    double *post = (double *)calloc(2 * Q * n, sizeof(double));
    if (!post)
        return -1;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t k = (size_t)y * nx + x;
            if (!mask[k])
                continue;
            double fp[2][Q];
            bad += collide_node(p, mask, f_in, rho_work, x, y, fp);
            for (int s = 0; s < 2; ++s)
                for (int i = 0; i < Q; ++i)
                    post[((size_t)s * Q + i) * n + k] = fp[s][i];
        }
    memset(f_out, 0, sizeof(double) * 2 * Q * n);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t k = (size_t)y * nx + x;
            if (!mask[k])
                continue;
            for (int s = 0; s < 2; ++s) {
                double dm = 0.0; /* mass returned beyond half-way bounce-back */
                for (int i = 0; i < Q; ++i) {
                    const double v = post[((size_t)s * Q + i) * n + k];
                    const int xn = x + CXI[i], yn = y + CYI[i];
                    if (node_is_fluid(p, mask, xn, yn)) {
                        f_out[((size_t)s * Q + i) * n + node_index(p, xn, yn)] = v;
                        continue;
                    }
                    const double q = orc_wall_fraction(p, x, y, i);
                    double back;
                    if (q < 0.5) {
                        const int xb = x - CXI[i], yb = y - CYI[i];
                        back = node_is_fluid(p, mask, xb, yb)
                                   ? 2.0 * q * v + (1.0 - 2.0 * q) *
                                         post[((size_t)s * Q + i) * n + node_index(p, xb, yb)]
                                   : v;
                    } else {
                        back = v / (2.0 * q) +
                               (1.0 - 1.0 / (2.0 * q)) * post[((size_t)s * Q + OPPOSITE[i]) * n + k];
                    }
                    f_out[((size_t)s * Q + OPPOSITE[i]) * n + k] = back;
                    dm += back - v;
                }
                /* Keep each species' mass: the difference goes back through the
                 * rest population, which carries no momentum (the rest
                 * population streams to the node itself and is already stored). */
                if (p->wall_interp == 1)
                    f_out[((size_t)s * Q + 0) * n + k] -= dm;
            }
        }
    free(post);
    return bad;
}

int orc_step(const orc_params *p, const uint8_t *mask, const double *f_in,
             double *f_out, double *rho_work)
{
    if (p->wall_interp)
        return orc_step_interp(p, mask, f_in, f_out, rho_work);
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    int bad = 0;

    orc_densities(p, mask, f_in, rho_work);
    memset(f_out, 0, sizeof(double) * 2 * Q * n);

#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const size_t k = (size_t)y * nx + x;
            if (!mask[k])
                continue;
            node_state st;
            gather_node(p, mask, f_in, rho_work, x, y, &st);
            if (!(st.rho[0] > 0.0) || !(st.rho[1] > 0.0) || !isfinite(st.rho[0] + st.rho[1]))
                ++bad;
            const double tau_mix = orc_tau_mix(p, st.rho[0], st.rho[1]);
            for (int s = 0; s < 2; ++s) {
                double fl[Q], feq_own[Q], feq_shift[Q], fneq[Q], fpost[Q];
                for (int i = 0; i < Q; ++i)
                    fl[i] = f_in[((size_t)s * Q + i) * n + k];
                /* Eq. 9: the force enters as a shift of the mixture velocity. */
                const double usx = st.ux + st.fx[s] / st.rho[s];
                const double usy = st.uy + st.fy[s] / st.rho[s];
                orc_equilibrium(st.rho[s], usx, usy, feq_shift);
                /* Eq. 6: the non-equilibrium momentum flux of component s is its
                 * flux minus that of its own local equilibrium, i.e. at its own
                 * velocity j^s / rho^s. */
                orc_equilibrium(st.rho[s], st.jx[s] / st.rho[s], st.jy[s] / st.rho[s], feq_own);
                if (p->reg_order == 3)
                    orc_regularize3(fl, feq_own, fneq, NULL);
                else
                    orc_regularize(fl, feq_own, fneq, NULL);
                for (int i = 0; i < Q; ++i)                      /* Eq. 3 */
                    fpost[i] = feq_shift[i] + (1.0 - 1.0 / tau_mix) * fneq[i];
                /* Eq. 1, left side: stream; half-way bounce-back at solid links. */
                for (int i = 0; i < Q; ++i) {
                    const int xn = x + CXI[i], yn = y + CYI[i];
                    if (node_is_fluid(p, mask, xn, yn))
                        f_out[((size_t)s * Q + i) * n + node_index(p, xn, yn)] = fpost[i];
                    else
                        f_out[((size_t)s * Q + OPPOSITE[i]) * n + k] = fpost[i];
                }
            }
        }
    }
    return bad;
}

/* Run nsteps steps in place on f (work: [2][9][n] + [2][n] doubles). Returns
 * the first step index whose input state had a bad node, or -1. */
int64_t orc_run(const orc_params *p, const uint8_t *mask, double *f, double *work, int64_t nsteps)
{
    const size_t n = (size_t)p->nx * p->ny;
    double *other = work;
    double *rho = work + 2 * Q * n;
    for (int64_t t = 0; t < nsteps; ++t) {
        const int bad = orc_step(p, mask, f, other, rho);
        memcpy(f, other, sizeof(double) * 2 * Q * n);
        if (bad)
            return t;
    }
    return -1;
}

/* ---- initial state: f_i = f_i^eq(rho0(x), 0) at fluid nodes ----------------- */
void orc_init(const orc_params *p, const uint8_t *mask, const double *rho0, double *f)
{
    const size_t n = (size_t)p->nx * p->ny;
    memset(f, 0, sizeof(double) * 2 * Q * n);
    for (int s = 0; s < 2; ++s)
        for (size_t k = 0; k < n; ++k) {
            if (!mask[k])
                continue;
            double feq[Q];
            orc_equilibrium(rho0[(size_t)s * n + k], 0.0, 0.0, feq);
            for (int i = 0; i < Q; ++i)
                f[((size_t)s * Q + i) * n + k] = feq[i];
        }
}

/* ---- macroscopic fields and monitors at time t ------------------------------
 * rho_out [2][n]: species densities.
 * u_out   [2][n]: physical mixture velocity u_mix + (F^o + F^w) / (2 rho).
 * p_out   [n]   : bulk pressure of the two-component mixture,
 *                 T0 (rho^o + rho^w) - G T0 rho^o rho^w.
 * mon     [8]   : sum rho^o, sum rho^w, sum of the physical momentum (x, y),
 *                 sum rho^o u_x, sum rho^o cos(2 pi x / nx),
 *                 sum rho^o sin(2 pi x / nx), number of bad nodes.
 * Solid nodes get 0 in every field.  Any output pointer may be NULL. */
void orc_moments(const orc_params *p, const uint8_t *mask, const double *f,
                 double *rho_work, double *rho_out, double *u_out, double *p_out,
                 double *mon)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    const double two_pi = 6.283185307179586476925286766559;
    double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    orc_densities(p, mask, f, rho_work);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t k = (size_t)y * nx + x;
            double r0 = 0, r1 = 0, ux = 0, uy = 0, pr = 0;
            if (mask[k]) {
                node_state st;
                gather_node(p, mask, f, rho_work, x, y, &st);
                const double rt = st.rho[0] + st.rho[1];
                const double px = st.jx[0] + st.jx[1] + 0.5 * (st.fx[0] + st.fx[1]);
                const double py = st.jy[0] + st.jy[1] + 0.5 * (st.fy[0] + st.fy[1]);
                r0 = st.rho[0];
                r1 = st.rho[1];
                ux = px / rt;
                uy = py / rt;
                pr = T0 * rt - p->G * T0 * r0 * r1;
                m[0] += r0;
                m[1] += r1;
                m[2] += px;
                m[3] += py;
                m[4] += r0 * ux;
                m[5] += r0 * cos(two_pi * x / nx);
                m[6] += r0 * sin(two_pi * x / nx);
                if (!(r0 > 0.0) || !(r1 > 0.0) || !isfinite(r0 + r1 + ux + uy))
                    m[7] += 1.0;
            }
            if (rho_out) {
                rho_out[k] = r0;
                rho_out[n + k] = r1;
            }
            if (u_out) {
                u_out[k] = ux;
                u_out[n + k] = uy;
            }
            if (p_out)
                p_out[k] = pr;
        }
    if (mon)
        for (int j = 0; j < 8; ++j)
            mon[j] = m[j];
}
