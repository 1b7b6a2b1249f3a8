/*
 * Plain FP64 CPU oracle of the relativistic particle-in-cell step of
 * Nattila, "Runko: Modern multiphysics toolbox for plasma simulations"
 * (arXiv 1906.06306).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or constant with the HIP
 * implementation.
 *
 * Everything is written on global (untiled) periodic arrays, in double
 * precision, in the order the paper's time-advance loop (Table 1) lists the
 * routines, without blocking, fusion or reordering.  Build with
 * -O2 -ffp-contract=off so that no multiply-add is contracted.
 *
 * Lattice (Sect. 2.3.1, the Yee staggering of the main text): storage index
 * (i,j,k) holds
 *   Ex at (i+1/2, j, k)     Ey at (i, j+1/2, k)     Ez at (i, j, k+1/2)
 *   Bx at (i, j+1/2, k+1/2) By at (i+1/2, j, k+1/2) Bz at (i+1/2, j+1/2, k)
 * J is co-located with E, the charge density rho sits on nodes (i,j,k).
 * Dimensions at or beyond D have extent 1; with periodic wrapping every
 * difference along them vanishes, which is the lower-dimensional lattice.
 * Field arrays are three planes of N = n0*n1*n2 values, x fastest.
 * Particle positions are global, in cell units, D values per particle
 * (plane per dimension); four-velocities u have 3 planes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t wrapi(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static int64_t cell(const int n[3], int64_t i, int64_t j, int64_t k)
{
    return wrapi(i, n[0]) + (int64_t)n[0] * (wrapi(j, n[1]) + (int64_t)n[1] * wrapi(k, n[2]));
}

static int64_t ncells(const int n[3]) { return (int64_t)n[0] * n[1] * n[2]; }

/* ---------------------------------------------------------------------- */
/* Field solver, Eqs. (fdE)/(fdB) with the forward/backward differences of
 * App. B, on the main-text lattice.                                       */

/* B <- B - h * curl(E), curl taken with forward differences so that each
 * B component lands on its own staggered point.  One half-step of the
 * split B advance of Table 1 uses h = c/2.                                */
void orc_advance_b(int D, const int n[3], double h, const double *E, double *B)
{
    (void)D;
    int64_t N = ncells(n);
    const double *Ex = E, *Ey = E + N, *Ez = E + 2 * N;
    double *Bx = B, *By = B + N, *Bz = B + 2 * N;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t c = cell(n, i, j, k);
                int64_t ip = cell(n, i + 1, j, k), jp = cell(n, i, j + 1, k), kp = cell(n, i, j, k + 1);
                double cx = (Ez[jp] - Ez[c]) - (Ey[kp] - Ey[c]);
                double cy = (Ex[kp] - Ex[c]) - (Ez[ip] - Ez[c]);
                double cz = (Ey[ip] - Ey[c]) - (Ex[jp] - Ex[c]);
                Bx[c] -= h * cx;
                By[c] -= h * cy;
                Bz[c] -= h * cz;
            }
}

/* E <- E + h * curl(B), backward differences.  push_e of Table 1 uses h=c. */
void orc_advance_e(int D, const int n[3], double h, const double *B, double *E)
{
    (void)D;
    int64_t N = ncells(n);
    const double *Bx = B, *By = B + N, *Bz = B + 2 * N;
    double *Ex = E, *Ey = E + N, *Ez = E + 2 * N;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t c = cell(n, i, j, k);
                int64_t im = cell(n, i - 1, j, k), jm = cell(n, i, j - 1, k), km = cell(n, i, j, k - 1);
                double cx = (Bz[c] - Bz[jm]) - (By[c] - By[km]);
                double cy = (Bx[c] - Bx[km]) - (Bz[c] - Bz[im]);
                double cz = (By[c] - By[im]) - (Bx[c] - Bx[jm]);
                Ex[c] += h * cx;
                Ey[c] += h * cy;
                Ez[c] += h * cz;
            }
}

/* add_cur of Table 1: E <- E - J (J already in field units, Eq. fdE). */
void orc_add_current(const int n[3], const double *J, double *E)
{
    int64_t M = 3 * ncells(n);
    for (int64_t m = 0; m < M; ++m) E[m] -= J[m];
}

/* ---------------------------------------------------------------------- */
/* Particles.                                                              */

/* staggering offset of field component comp (0..2 = E, 3..5 = B) along d */
static double stagger(int comp, int d)
{
    static const double off[6][3] = {
        {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
        {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0},
    };
    return off[comp][d];
}

/* Linear ("volume averaging") interpolation, Sect. 2.3.2: every component
 * is interpolated from its own staggered sub-lattice with first-order
 * (cloud-in-cell) weights over the 2^D surrounding points.
 * x: D planes of np global positions.  Out: 3 planes each of Ep, Bp.      */
void orc_interp(int D, const int n[3], const double *E, const double *B,
                int64_t np, const double *x, double *Ep, double *Bp)
{
    int64_t N = ncells(n);
    for (int64_t p = 0; p < np; ++p) {
        for (int comp = 0; comp < 6; ++comp) {
            const double *F = comp < 3 ? E + comp * N : B + (comp - 3) * N;
            int64_t base[3] = {0, 0, 0};
            double w[3] = {0.0, 0.0, 0.0};
            for (int d = 0; d < D; ++d) {
                double xi = x[d * np + p] - stagger(comp, d);
                double fl = floor(xi);
                base[d] = (int64_t)fl;
                w[d] = xi - fl;
            }
            double acc = 0.0;
            int ncorner = 1 << D;
            for (int cn = 0; cn < ncorner; ++cn) {
                int64_t idx[3] = {base[0], base[1], base[2]};
                double wt = 1.0;
                for (int d = 0; d < D; ++d) {
                    int bit = (cn >> d) & 1;
                    idx[d] += bit;
                    wt *= bit ? w[d] : 1.0 - w[d];
                }
                acc += wt * F[cell(n, idx[0], idx[1], idx[2])];
            }
            if (comp < 3) Ep[comp * np + p] = acc;
            else Bp[(comp - 3) * np + p] = acc;
        }
    }
}

/* Relativistic Boris velocity update, App. C.  Velocities are carried in
 * units of the Courant number c inside the update (u' = c u).
 * s = q/(m m_pm), the species charge-to-mass factor of App. C.
 * u: 3 planes, updated in place from u^{n-1/2} to u^{n+1/2}.              */
void orc_boris(int64_t np, double c, double s, const double *Ep, const double *Bp, double *u)
{
    for (int64_t p = 0; p < np; ++p) {
        double ex = 0.5 * s * Ep[p], ey = 0.5 * s * Ep[np + p], ez = 0.5 * s * Ep[2 * np + p];
        /* first half of the electric kick */
        double u1x = c * u[p] + ex, u1y = c * u[np + p] + ey, u1z = c * u[2 * np + p] + ez;
        double g1 = sqrt(1.0 + (u1x * u1x + u1y * u1y + u1z * u1z) / (c * c));
        /* rotation vector t = s B / (2 c gamma_1) and f = 2/(1+|t|^2) */
        double tx = s * Bp[p] / (2.0 * c * g1);
        double ty = s * Bp[np + p] / (2.0 * c * g1);
        double tz = s * Bp[2 * np + p] / (2.0 * c * g1);
        double f = 2.0 / (1.0 + (tx * tx + ty * ty + tz * tz));
        /* u2' = f (u1' + u1' x t) */
        double u2x = f * (u1x + (u1y * tz - u1z * ty));
        double u2y = f * (u1y + (u1z * tx - u1x * tz));
        double u2z = f * (u1z + (u1x * ty - u1y * tx));
        /* u3' = u1' + u2' x t + second half of the electric kick */
        double u3x = u1x + (u2y * tz - u2z * ty) + ex;
        double u3y = u1y + (u2z * tx - u2x * tz) + ey;
        double u3z = u1z + (u2x * ty - u2y * tx) + ez;
        u[p] = u3x / c;
        u[np + p] = u3y / c;
        u[2 * np + p] = u3z / c;
    }
}

/* Position advance, Eq. (fdX): dx = c u / gamma with gamma of u^{n+1/2}.
 * All three displacement components are returned in disp (3 planes); the
 * D grid coordinates of x are advanced in place (no wrapping here).       */
void orc_move(int D, int64_t np, double c, const double *u, double *x, double *disp)
{
    for (int64_t p = 0; p < np; ++p) {
        double ux = u[p], uy = u[np + p], uz = u[2 * np + p];
        double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        double dv[3] = {c * ux / g, c * uy / g, c * uz / g};
        for (int m = 0; m < 3; ++m) disp[m * np + p] = dv[m];
        for (int d = 0; d < D; ++d) x[d * np + p] += dv[d];
    }
}

/* Deposit one zigzag segment: flux F (3 comps), weight W, displacement dv
 * and cell i along the grid dimensions.  A segment is a straight move inside
 * one cell, so its current is the path average of the first-order particle
 * shape.  Component m goes to J_m at the cell index along m and, along every
 * other grid dimension d, to the two points i_d, i_d+1 with the linear
 * weights 1-W_d and W_d evaluated at the segment midpoint.  When two such
 * transverse dimensions a, b exist, the path average of the product of the
 * two linear factors adds sigma_a sigma_b dv_a dv_b / 12 (sigma = -1 at the
 * lower point, +1 at the upper point); without it the deposit would not
 * satisfy the discrete continuity equation in 3D.                        */
static void deposit_segment(int D, const int n[3], double *J, const double F[3],
                            const double W[3], const double dv[3], const int64_t i[3])
{
    int64_t N = ncells(n);
    for (int m = 0; m < 3; ++m) {
        int ntrans = 0;
        for (int d = 0; d < D; ++d) ntrans += (d != m);
        int ncorner = 1 << D;
        for (int cn = 0; cn < ncorner; ++cn) {
            /* corners along dimension m itself do not exist */
            if (m < D && ((cn >> m) & 1)) continue;
            int64_t idx[3] = {i[0], i[1], i[2]};
            double wt = 1.0, cross = 1.0;
            for (int d = 0; d < D; ++d) {
                if (d == m) continue;
                int bit = (cn >> d) & 1;
                idx[d] += bit;
                wt *= bit ? W[d] : 1.0 - W[d];
                cross *= bit ? dv[d] : -dv[d];
            }
            if (ntrans == 2) wt += cross / 12.0;
            J[m * N + cell(n, idx[0], idx[1], idx[2])] += F[m] * wt;
        }
    }
}

/* Charge-conserving ZigZag deposit, App. D (after Umeda et al. 2003), of
 * every particle moving from x1 to x2 (D planes each, unwrapped) with
 * charge q.  disp holds the three displacement components; the ones along
 * non-grid dimensions are split evenly over the two segments (relay point
 * at the midpoint).  J is accumulated (not cleared) with periodic wrap.   */
void orc_zigzag(int D, const int n[3], double q, int64_t np, const double *x1,
                const double *x2, const double *disp, double *J)
{
    for (int64_t p = 0; p < np; ++p) {
        double F1[3], F2[3], W1[3] = {0, 0, 0}, W2[3] = {0, 0, 0};
        double d1[3] = {0, 0, 0}, d2[3] = {0, 0, 0};
        int64_t i1[3] = {0, 0, 0}, i2[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            if (d < D) {
                double a = x1[d * np + p], b = x2[d * np + p];
                double fa = floor(a), fb = floor(b);
                double lo = fa < fb ? fa : fb, hi = fa > fb ? fa : fb;
                double mid = 0.5 * (a + b);
                double inner = hi > mid ? hi : mid;      /* max{max{i1,i2}, mid} */
                double xr = (lo + 1.0) < inner ? (lo + 1.0) : inner; /* min{min{i1,i2}+1, .} */
                F1[d] = q * (xr - a);
                F2[d] = q * (b - xr);
                W1[d] = 0.5 * (a + xr) - fa;
                W2[d] = 0.5 * (b + xr) - fb;
                d1[d] = xr - a;
                d2[d] = b - xr;
                i1[d] = (int64_t)fa;
                i2[d] = (int64_t)fb;
            } else {
                double h = 0.5 * disp[d * np + p];
                F1[d] = q * h;
                F2[d] = q * h;
            }
        }
        deposit_segment(D, n, J, F1, W1, d1, i1);
        deposit_segment(D, n, J, F2, W2, d2, i2);
    }
}

/* Periodic wrap into [0, n): a result that rounds up to n becomes 0. */
void orc_wrap(int D, const int n[3], int64_t np, double *x)
{
    for (int d = 0; d < D; ++d) {
        double L = (double)n[d];
        for (int64_t p = 0; p < np; ++p) {
            double v = x[d * np + p];
            if (v < 0.0) v += L;
            else if (v >= L) v -= L;
            if (v >= L) v = 0.0;
            x[d * np + p] = v;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* One full time step, routines in the order of Table 1:
 *   push_half_b1; interp_em + push (every species); push_half_b2; push_e;
 *   comp_curr (every species, J cleared first); the particle
 *   communication rows, which on one periodic domain reduce to wrapping the
 *   positions; add_cur.
 * Species s has n_per[s] particles, positions x[s] (D planes, global) and
 * four-velocities u[s] (3 planes); q[s] is its charge, sgn[s] its App. C
 * factor s.  J is overwritten with this step's current.  Returns 0, or -1
 * if scratch memory could not be allocated.                               */
int orc_step(int D, const int n[3], double c, int nspecies, const int64_t *n_per,
             double **x, double **u, const double *q, const double *sgn,
             double *E, double *B, double *J)
{
    int64_t N = ncells(n);
    double **xold = calloc((size_t)nspecies, sizeof(double *));
    double **disp = calloc((size_t)nspecies, sizeof(double *));
    int64_t npmax = 1;
    for (int s = 0; s < nspecies; ++s) npmax = n_per[s] > npmax ? n_per[s] : npmax;
    double *fp = malloc(sizeof(double) * 6 * (size_t)npmax);
    int ok = xold && disp && fp;
    for (int s = 0; ok && s < nspecies; ++s) {
        xold[s] = malloc(sizeof(double) * (size_t)(D * n_per[s] + 1));
        disp[s] = malloc(sizeof(double) * (size_t)(3 * n_per[s] + 1));
        ok = xold[s] && disp[s];
    }
    if (ok) {
        orc_advance_b(D, n, 0.5 * c, E, B);                       /* push_half_b1 */
        for (int s = 0; s < nspecies; ++s) {                       /* interp_em, push */
            int64_t np = n_per[s];
            memcpy(xold[s], x[s], sizeof(double) * (size_t)(D * np));
            orc_interp(D, n, E, B, np, x[s], fp, fp + 3 * np);
            orc_boris(np, c, sgn[s], fp, fp + 3 * np, u[s]);
            orc_move(D, np, c, u[s], x[s], disp[s]);
        }
        orc_advance_b(D, n, 0.5 * c, E, B);                       /* push_half_b2 */
        orc_advance_e(D, n, c, B, E);                             /* push_e */
        memset(J, 0, sizeof(double) * 3 * (size_t)N);             /* comp_curr */
        for (int s = 0; s < nspecies; ++s)
            orc_zigzag(D, n, q[s], n_per[s], xold[s], x[s], disp[s], J);
        for (int s = 0; s < nspecies; ++s) orc_wrap(D, n, n_per[s], x[s]);
        orc_add_current(n, J, E);                                 /* add_cur */
    }
    for (int s = 0; xold && disp && s < nspecies; ++s) {
        free(xold[s]);
        free(disp[s]);
    }
    free(xold);
    free(disp);
    free(fp);
    return ok ? 0 : -1;
}

/* ---------------------------------------------------------------------- */
/* Diagnostics (the paper prints no formula; these follow from App. B).   */

/* Charge density on nodes: cloud-in-cell weights of each particle times q.
 * rho is accumulated (not cleared). */
void orc_rho(int D, const int n[3], double q, int64_t np, const double *x, double *rho)
{
    for (int64_t p = 0; p < np; ++p) {
        int64_t base[3] = {0, 0, 0};
        double w[3] = {0, 0, 0};
        for (int d = 0; d < D; ++d) {
            double fl = floor(x[d * np + p]);
            base[d] = (int64_t)fl;
            w[d] = x[d * np + p] - fl;
        }
        for (int cn = 0; cn < (1 << D); ++cn) {
            int64_t idx[3] = {base[0], base[1], base[2]};
            double wt = 1.0;
            for (int d = 0; d < D; ++d) {
                int bit = (cn >> d) & 1;
                idx[d] += bit;
                wt *= bit ? w[d] : 1.0 - w[d];
            }
            rho[cell(n, idx[0], idx[1], idx[2])] += q * wt;
        }
    }
}

/* Backward-difference divergence of an E-like (edge) field, on nodes. */
void orc_div_edge(const int n[3], const double *F, double *out)
{
    int64_t N = ncells(n);
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t c = cell(n, i, j, k);
                out[c] = (F[c] - F[cell(n, i - 1, j, k)]) + (F[N + c] - F[N + cell(n, i, j - 1, k)]) +
                         (F[2 * N + c] - F[2 * N + cell(n, i, j, k - 1)]);
            }
}

/* Forward-difference divergence of a B-like (face) field, on cell centres. */
void orc_div_face(const int n[3], const double *F, double *out)
{
    int64_t N = ncells(n);
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t c = cell(n, i, j, k);
                out[c] = (F[cell(n, i + 1, j, k)] - F[c]) + (F[N + cell(n, i, j + 1, k)] - F[N + c]) +
                         (F[2 * N + cell(n, i, j, k + 1)] - F[2 * N + c]);
            }
}

/* Field energy 1/2 sum(E^2 + B^2) and kinetic energy sum m c^2 (gamma-1). */
double orc_field_energy(const int n[3], const double *E, const double *B)
{
    int64_t M = 3 * ncells(n);
    double s = 0.0;
    for (int64_t m = 0; m < M; ++m) s += E[m] * E[m] + B[m] * B[m];
    return 0.5 * s;
}

double orc_kinetic_energy(int64_t np, double mass, double c, const double *u)
{
    double s = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        double g = sqrt(1.0 + u[p] * u[p] + u[np + p] * u[np + p] + u[2 * np + p] * u[2 * np + p]);
        s += g - 1.0;
    }
    return mass * c * c * s;
}

/* ====================================================================== */
/* Conducting, reflecting walls in x (the shock configuration; the paper
 * names reflecting walls for its shock runs but gives no boundary
 * formulas, so this is the reading used throughout this implementation).
 *
 * The walls sit on the node planes x = 0 and x = n0; y and z stay
 * periodic.  Tangential E (Ey, Ez) and normal B (Bx) vanish on the wall
 * planes; storage node i = 0 holds the x = 0 plane and also stands for the
 * x = n0 plane (which the periodic storage maps onto it), so both are held
 * at zero.  Components staggered by 1/2 in x (Ex, By, Bz) see the wall as a
 * mirror: their value at -1/2 equals the one at +1/2, and the one at
 * n0 + 1/2 the one at n0 - 1/2.  A particle whose move crosses a wall is
 * reflected (x -> -x or 2 n0 - x, u_x -> -u_x) and deposits its current
 * along the broken path: x^n to the wall point, then the wall point to the
 * reflected position, each piece by the ZigZag rule, which keeps the
 * discrete continuity equation exact.                                      */

static double wall_value(const int n[3], const double *F, int comp, int64_t i, int64_t j, int64_t k)
{
    if (stagger(comp, 0) > 0.0) {
        /* mirror images of the half-integer sub-lattice */
        if (i < 0) i = -1 - i;
        if (i >= n[0]) i = 2 * (int64_t)n[0] - 1 - i;
    } else if (i == 0 || i == n[0]) {
        /* node-centred in x on a wall plane: Ey, Ez, Bx are zero there */
        return 0.0;
    }
    return F[cell(n, i, j, k)];
}

/* interp_em with the wall images (otherwise as orc_interp) */
void orc_interp_walls(int D, const int n[3], const double *E, const double *B, int64_t np, const double *x,
                         double *Ep, double *Bp)
{
    int64_t N = ncells(n);
    for (int64_t p = 0; p < np; ++p) {
        for (int comp = 0; comp < 6; ++comp) {
            const double *F = comp < 3 ? E + comp * N : B + (comp - 3) * N;
            int64_t base[3] = {0, 0, 0};
            double w[3] = {0.0, 0.0, 0.0};
            for (int d = 0; d < D; ++d) {
                double xi = x[d * np + p] - stagger(comp, d);
                double fl = floor(xi);
                base[d] = (int64_t)fl;
                w[d] = xi - fl;
            }
            double acc = 0.0;
            for (int cn = 0; cn < (1 << D); ++cn) {
                int64_t idx[3] = {base[0], base[1], base[2]};
                double wt = 1.0;
                for (int d = 0; d < D; ++d) {
                    int bit = (cn >> d) & 1;
                    idx[d] += bit;
                    wt *= bit ? w[d] : 1.0 - w[d];
                }
                acc += wt * wall_value(n, F, comp, idx[0], idx[1], idx[2]);
            }
            if (comp < 3) Ep[comp * np + p] = acc;
            else Bp[(comp - 3) * np + p] = acc;
        }
    }
}

/* ZigZag deposit (App. D) of one straight move a -> b (grid dimensions)
 * with displacement dnon along the non-grid dimensions. */
static void zigzag_path(int D, const int n[3], double q, const double a[3], const double b[3],
                        const double dnon[3], double *J)
{
    double F1[3], F2[3], W1[3] = {0, 0, 0}, W2[3] = {0, 0, 0};
    double d1[3] = {0, 0, 0}, d2[3] = {0, 0, 0};
    int64_t i1[3] = {0, 0, 0}, i2[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        if (d < D) {
            double fa = floor(a[d]), fb = floor(b[d]);
            double lo = fa < fb ? fa : fb, hi = fa > fb ? fa : fb;
            double mid = 0.5 * (a[d] + b[d]);
            double inner = hi > mid ? hi : mid;
            double xr = (lo + 1.0) < inner ? (lo + 1.0) : inner;
            F1[d] = q * (xr - a[d]);
            F2[d] = q * (b[d] - xr);
            W1[d] = 0.5 * (a[d] + xr) - fa;
            W2[d] = 0.5 * (b[d] + xr) - fb;
            d1[d] = xr - a[d];
            d2[d] = b[d] - xr;
            i1[d] = (int64_t)fa;
            i2[d] = (int64_t)fb;
        } else {
            F1[d] = q * 0.5 * dnon[d];
            F2[d] = q * 0.5 * dnon[d];
        }
    }
    deposit_segment(D, n, J, F1, W1, d1, i1);
    deposit_segment(D, n, J, F2, W2, d2, i2);
}

/* The largest double below v (v > 0). */
static double below(double v) { return nextafter(v, 0.0); }

/* One full step with walls in x, in the order of orc_step.  Positions must
 * start inside [0, n0); E, B with the wall planes at zero (Ey, Ez, Bx at
 * i = 0).  Returns 0, or -1 if scratch memory could not be allocated.     */
int orc_step_walls(int D, const int n[3], double c, int nspecies, const int64_t *n_per,
                   double **x, double **u, const double *q, const double *sgn,
                   double *E, double *B, double *J)
{
    if (nspecies < 1) return -1;
    int64_t N = ncells(n);
    double L = (double)n[0];
    int64_t npmax = 1;
    for (int s = 0; s < nspecies; ++s) npmax = n_per[s] > npmax ? n_per[s] : npmax;
    double *fp = malloc(sizeof(double) * 6 * (size_t)npmax);
    if (!fp) return -1;
    double **xold = calloc((size_t)nspecies, sizeof(double *));
    double **disp = calloc((size_t)nspecies, sizeof(double *));
    int ok = xold && disp;
    for (int s = 0; ok && s < nspecies; ++s) {
        xold[s] = malloc(sizeof(double) * (size_t)(D * n_per[s] + 1));
        disp[s] = malloc(sizeof(double) * (size_t)(3 * n_per[s] + 1));
        ok = xold[s] && disp[s];
    }
    if (ok) {
        orc_advance_b(D, n, 0.5 * c, E, B);                       /* push_half_b1 */
        for (int s = 0; s < nspecies; ++s) {                       /* interp_em, push */
            int64_t np = n_per[s];
            memcpy(xold[s], x[s], sizeof(double) * (size_t)(D * np));
            orc_interp_walls(D, n, E, B, np, x[s], fp, fp + 3 * np);
            orc_boris(np, c, sgn[s], fp, fp + 3 * np, u[s]);
            orc_move(D, np, c, u[s], x[s], disp[s]);
        }
        orc_advance_b(D, n, 0.5 * c, E, B);                       /* push_half_b2 */
        orc_advance_e(D, n, c, B, E);                             /* push_e */
        memset(J, 0, sizeof(double) * 3 * (size_t)N);             /* comp_curr */
        for (int s = 0; s < nspecies; ++s) {
            int64_t np = n_per[s];
            for (int64_t p = 0; p < np; ++p) {
                double a[3] = {0, 0, 0}, b[3] = {0, 0, 0}, dn[3] = {0, 0, 0};
                for (int d = 0; d < D; ++d) {
                    a[d] = xold[s][d * np + p];
                    b[d] = x[s][d * np + p];
                }
                for (int m = D; m < 3; ++m) dn[m] = disp[s][m * np + p];
                double bx = b[0];
                if (bx >= 0.0 && bx < L) {
                    zigzag_path(D, n, q[s], a, b, dn, J);
                    continue;
                }
                /* reflection: wall point at fraction t of the move */
                double wx = bx < 0.0 ? 0.0 : L;
                double t = (wx - a[0]) / (bx - a[0]);
                double w[3] = {wx, 0, 0}, r[3] = {0, 0, 0}, dn1[3] = {0, 0, 0}, dn2[3] = {0, 0, 0};
                for (int d = 1; d < D; ++d) w[d] = a[d] + t * (b[d] - a[d]);
                for (int m = D; m < 3; ++m) {
                    dn1[m] = t * dn[m];
                    dn2[m] = dn[m] - dn1[m];
                }
                r[0] = bx < 0.0 ? -bx : 2.0 * L - bx;
                if (r[0] >= L) r[0] = below(L);
                for (int d = 1; d < D; ++d) r[d] = b[d];
                zigzag_path(D, n, q[s], a, w, dn1, J);
                zigzag_path(D, n, q[s], w, r, dn2, J);
                x[s][p] = r[0];
                u[s][p] = -u[s][p];
            }
        }
        /* particle communication: periodic wrap along y and z only */
        for (int s = 0; s < nspecies; ++s)
            for (int d = 1; d < D; ++d) {
                double Ld = (double)n[d];
                for (int64_t p = 0; p < n_per[s]; ++p) {
                    double v = x[s][d * n_per[s] + p];
                    if (v < 0.0) v += Ld;
                    else if (v >= Ld) v -= Ld;
                    if (v >= Ld) v = 0.0;
                    x[s][d * n_per[s] + p] = v;
                }
            }
        orc_add_current(n, J, E);                                 /* add_cur */
        /* the wall planes: tangential E and normal B vanish */
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j) {
                int64_t cw = cell(n, 0, j, k);
                E[N + cw] = 0.0;
                E[2 * N + cw] = 0.0;
                B[cw] = 0.0;
            }
    }
    for (int s = 0; xold && disp && s < nspecies; ++s) {
        free(xold[s]);
        free(disp[s]);
    }
    free(xold);
    free(disp);
    free(fp);
    return ok ? 0 : -1;
}

/* ====================================================================== */
/* Solvers the paper lists beside the Boris pusher and the plain current
 * (its table of modules and solvers): the Vay and Higuera-Cary pushers and
 * the 3-point binomial current filter, written from their published
 * definitions in the units of App. C (velocities w = c u inside an update,
 * half electric kick eps = s E / 2, rotation vector tau = s B / (2 c), so
 * that Boris uses t = tau / gamma_1).                                     */

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Lorentz factor of the implicit rotation: the gamma that solves
 * w1 = w' + (w1 / gamma) x tau, from gamma'^2 = 1 + |w'|^2/c^2 and
 * u* = w'.tau / c (Vay 2008; Higuera and Cary 2017). */
static double implicit_gamma(const double wp[3], const double tau[3], double c)
{
    double g2 = 1.0 + dot3(wp, wp) / (c * c);
    double us = dot3(wp, tau) / c;
    double t2 = dot3(tau, tau);
    double sig = g2 - t2;
    return sqrt(0.5 * (sig + sqrt(sig * sig + 4.0 * (t2 + us * us))));
}

/* w <- s (w + (w.t) t + w x t), s = 1/(1+|t|^2) */
static void exact_rotation(const double w[3], const double t[3], double o[3])
{
    double wt = dot3(w, t), sf = 1.0 / (1.0 + dot3(t, t)), x[3];
    cross3(w, t, x);
    for (int i = 0; i < 3; ++i) o[i] = sf * (w[i] + wt * t[i] + x[i]);
}

/* Vay pusher: the full electric kick and half the magnetic kick with the old
 * velocity, then the other magnetic half with the new velocity, solved
 * exactly for its Lorentz factor. */
void orc_vay(int64_t np, double c, double s, const double *Ep, const double *Bp, double *u)
{
    for (int64_t p = 0; p < np; ++p) {
        double w0[3], tau[3], wp[3], vt[3], t[3], w1[3];
        for (int i = 0; i < 3; ++i) {
            w0[i] = c * u[i * np + p];
            tau[i] = s * Bp[i * np + p] / (2.0 * c);
        }
        double g0 = sqrt(1.0 + dot3(w0, w0) / (c * c));
        double v0[3] = {w0[0] / g0, w0[1] / g0, w0[2] / g0};
        cross3(v0, tau, vt);
        for (int i = 0; i < 3; ++i) wp[i] = w0[i] + s * Ep[i * np + p] + vt[i];
        double g1 = implicit_gamma(wp, tau, c);
        for (int i = 0; i < 3; ++i) t[i] = tau[i] / g1;
        exact_rotation(wp, t, w1);
        for (int i = 0; i < 3; ++i) u[i * np + p] = w1[i] / c;
    }
}

/* Higuera-Cary pusher: Boris's split (half kick, rotation, half kick) with
 * the rotation's Lorentz factor taken from the implicit (volume-preserving)
 * relation instead of gamma_1. */
void orc_hc(int64_t np, double c, double s, const double *Ep, const double *Bp, double *u)
{
    for (int64_t p = 0; p < np; ++p) {
        double eps[3], tau[3], wm[3], t[3], wpl[3], x[3];
        for (int i = 0; i < 3; ++i) {
            eps[i] = 0.5 * s * Ep[i * np + p];
            tau[i] = s * Bp[i * np + p] / (2.0 * c);
            wm[i] = c * u[i * np + p] + eps[i];
        }
        double g = implicit_gamma(wm, tau, c);
        for (int i = 0; i < 3; ++i) t[i] = tau[i] / g;
        exact_rotation(wm, t, wpl);
        cross3(wpl, t, x);
        for (int i = 0; i < 3; ++i) u[i * np + p] = (wpl[i] + eps[i] + x[i]) / c;
    }
}

/* Binomial current filter: each pass replaces every value by
 * (F[i-1] + 2 F[i] + F[i+1]) / 4 along every grid dimension in turn
 * (periodic), on nplanes planes of the field. */
int orc_filter_binomial(int D, const int n[3], int passes, int nplanes, double *F)
{
    int64_t N = ncells(n);
    double *tmp = malloc(sizeof(double) * (size_t)N);
    if (!tmp) return -1;
    for (int pass = 0; pass < passes; ++pass)
        for (int m = 0; m < nplanes; ++m) {
            double *P = F + m * N;
            for (int d = 0; d < D; ++d) {
                for (int k = 0; k < n[2]; ++k)
                    for (int j = 0; j < n[1]; ++j)
                        for (int i = 0; i < n[0]; ++i) {
                            int64_t lo = d == 0 ? cell(n, i - 1, j, k) : d == 1 ? cell(n, i, j - 1, k) : cell(n, i, j, k - 1);
                            int64_t hi = d == 0 ? cell(n, i + 1, j, k) : d == 1 ? cell(n, i, j + 1, k) : cell(n, i, j, k + 1);
                            int64_t c0 = cell(n, i, j, k);
                            tmp[c0] = 0.25 * P[lo] + 0.5 * P[c0] + 0.25 * P[hi];
                        }
                memcpy(P, tmp, sizeof(double) * (size_t)N);
            }
        }
    free(tmp);
    return 0;
}

/* Fourth-order FDTD (the solver table's FDTD4): every difference of the
 * curls spans the staggered points at +-1/2 and +-3/2 with the weights 9/8
 * and -1/24, e.g. forward D f(i) = 9/8 (f(i+1) - f(i)) - 1/24 (f(i+2) -
 * f(i-1)), backward D f(i) = 9/8 (f(i) - f(i-1)) - 1/24 (f(i+1) - f(i-2)).
 * These are combinations of single- and triple-cell differences, so the
 * lattice divergences still annihilate the curls. */
static double d4p(const double *F, const int n[3], int axis, int i, int j, int k)
{
    int o[3] = {0, 0, 0};
    o[axis] = 1;
    double f0 = F[cell(n, i, j, k)];
    double f1 = F[cell(n, i + o[0], j + o[1], k + o[2])];
    double f2 = F[cell(n, i + 2 * o[0], j + 2 * o[1], k + 2 * o[2])];
    double fm = F[cell(n, i - o[0], j - o[1], k - o[2])];
    return 9.0 / 8.0 * (f1 - f0) - 1.0 / 24.0 * (f2 - fm);
}

static double d4m(const double *F, const int n[3], int axis, int i, int j, int k)
{
    int o[3] = {0, 0, 0};
    o[axis] = 1;
    double f0 = F[cell(n, i, j, k)];
    double fm = F[cell(n, i - o[0], j - o[1], k - o[2])];
    double fm2 = F[cell(n, i - 2 * o[0], j - 2 * o[1], k - 2 * o[2])];
    double f1 = F[cell(n, i + o[0], j + o[1], k + o[2])];
    return 9.0 / 8.0 * (f0 - fm) - 1.0 / 24.0 * (f1 - fm2);
}

/* B <- B - h curl+ E with the fourth-order differences. */
void orc_advance_b4(int D, const int n[3], double h, const double *E, double *B)
{
    (void)D;
    int64_t N = ncells(n);
    const double *Ex = E, *Ey = E + N, *Ez = E + 2 * N;
    double *Bx = B, *By = B + N, *Bz = B + 2 * N;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t c = cell(n, i, j, k);
                double cx = d4p(Ez, n, 1, i, j, k) - d4p(Ey, n, 2, i, j, k);
                double cy = d4p(Ex, n, 2, i, j, k) - d4p(Ez, n, 0, i, j, k);
                double cz = d4p(Ey, n, 0, i, j, k) - d4p(Ex, n, 1, i, j, k);
                Bx[c] -= h * cx;
                By[c] -= h * cy;
                Bz[c] -= h * cz;
            }
}

/* E <- E + h curl- B with the fourth-order differences. */
void orc_advance_e4(int D, const int n[3], double h, const double *B, double *E)
{
    (void)D;
    int64_t N = ncells(n);
    const double *Bx = B, *By = B + N, *Bz = B + 2 * N;
    double *Ex = E, *Ey = E + N, *Ez = E + 2 * N;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t c = cell(n, i, j, k);
                double cx = d4m(Bz, n, 1, i, j, k) - d4m(By, n, 2, i, j, k);
                double cy = d4m(Bx, n, 2, i, j, k) - d4m(Bz, n, 0, i, j, k);
                double cz = d4m(By, n, 0, i, j, k) - d4m(Bx, n, 1, i, j, k);
                Ex[c] += h * cx;
                Ey[c] += h * cy;
                Ez[c] += h * cz;
            }
}

/* One full step with the options the solver table allows: walls in x
 * (walls = 1, see orc_step_walls), the pusher (0 Boris, 1 Vay,
 * 2 Higuera-Cary), the number of binomial filter passes applied to the
 * current after comp_curr and before add_cur, and the FDTD order (2, or 4
 * for FDTD4).  With walls = 0, pusher = 0, passes = 0 and order 2 it is
 * orc_step; with walls = 1, orc_step_walls.                               */
int orc_step_opts(int D, const int n[3], double c, int nspecies, const int64_t *n_per,
                  double **x, double **u, const double *q, const double *sgn,
                  double *E, double *B, double *J, int walls, int pusher, int passes, int order)
{
    if (nspecies < 1) return -1;
    int64_t N = ncells(n);
    double L = (double)n[0];
    int64_t npmax = 1;
    for (int s = 0; s < nspecies; ++s) npmax = n_per[s] > npmax ? n_per[s] : npmax;
    double *fp = malloc(sizeof(double) * 6 * (size_t)npmax);
    if (!fp) return -1;
    double **xold = calloc((size_t)nspecies, sizeof(double *));
    double **disp = calloc((size_t)nspecies, sizeof(double *));
    int ok = xold && disp;
    for (int s = 0; ok && s < nspecies; ++s) {
        xold[s] = malloc(sizeof(double) * (size_t)(D * n_per[s] + 1));
        disp[s] = malloc(sizeof(double) * (size_t)(3 * n_per[s] + 1));
        ok = xold[s] && disp[s];
    }
    if (ok) {
        void (*adv_b)(int, const int *, double, const double *, double *) = order == 4 ? orc_advance_b4 : orc_advance_b;
        void (*adv_e)(int, const int *, double, const double *, double *) = order == 4 ? orc_advance_e4 : orc_advance_e;
        adv_b(D, n, 0.5 * c, E, B);                               /* push_half_b1 */
        for (int s = 0; s < nspecies; ++s) {                       /* interp_em, push */
            int64_t np = n_per[s];
            memcpy(xold[s], x[s], sizeof(double) * (size_t)(D * np));
            if (walls) orc_interp_walls(D, n, E, B, np, x[s], fp, fp + 3 * np);
            else orc_interp(D, n, E, B, np, x[s], fp, fp + 3 * np);
            if (pusher == 1) orc_vay(np, c, sgn[s], fp, fp + 3 * np, u[s]);
            else if (pusher == 2) orc_hc(np, c, sgn[s], fp, fp + 3 * np, u[s]);
            else orc_boris(np, c, sgn[s], fp, fp + 3 * np, u[s]);
            orc_move(D, np, c, u[s], x[s], disp[s]);
        }
        adv_b(D, n, 0.5 * c, E, B);                               /* push_half_b2 */
        adv_e(D, n, c, B, E);                                     /* push_e */
        memset(J, 0, sizeof(double) * 3 * (size_t)N);             /* comp_curr */
        for (int s = 0; s < nspecies; ++s) {
            int64_t np = n_per[s];
            if (!walls) {
                orc_zigzag(D, n, q[s], np, xold[s], x[s], disp[s], J);
                continue;
            }
            for (int64_t p = 0; p < np; ++p) {
                double a[3] = {0, 0, 0}, b[3] = {0, 0, 0}, dn[3] = {0, 0, 0};
                for (int d = 0; d < D; ++d) {
                    a[d] = xold[s][d * np + p];
                    b[d] = x[s][d * np + p];
                }
                for (int m = D; m < 3; ++m) dn[m] = disp[s][m * np + p];
                double bx = b[0];
                if (bx >= 0.0 && bx < L) {
                    zigzag_path(D, n, q[s], a, b, dn, J);
                    continue;
                }
                double wx = bx < 0.0 ? 0.0 : L;
                double t = (wx - a[0]) / (bx - a[0]);
                double w[3] = {wx, 0, 0}, r[3] = {0, 0, 0}, dn1[3] = {0, 0, 0}, dn2[3] = {0, 0, 0};
                for (int d = 1; d < D; ++d) w[d] = a[d] + t * (b[d] - a[d]);
                for (int m = D; m < 3; ++m) {
                    dn1[m] = t * dn[m];
                    dn2[m] = dn[m] - dn1[m];
                }
                r[0] = bx < 0.0 ? -bx : 2.0 * L - bx;
                if (r[0] >= L) r[0] = below(L);
                for (int d = 1; d < D; ++d) r[d] = b[d];
                zigzag_path(D, n, q[s], a, w, dn1, J);
                zigzag_path(D, n, q[s], w, r, dn2, J);
                x[s][p] = r[0];
                u[s][p] = -u[s][p];
            }
        }
        /* particle communication: periodic wrap (y and z only with walls) */
        for (int s = 0; s < nspecies; ++s)
            for (int d = walls ? 1 : 0; d < D; ++d) {
                double Ld = (double)n[d];
                for (int64_t p = 0; p < n_per[s]; ++p) {
                    double v = x[s][d * n_per[s] + p];
                    if (v < 0.0) v += Ld;
                    else if (v >= Ld) v -= Ld;
                    if (v >= Ld) v = 0.0;
                    x[s][d * n_per[s] + p] = v;
                }
            }
        if (passes > 0 && orc_filter_binomial(D, n, passes, 3, J) != 0) ok = 0;
        if (ok) {
            orc_add_current(n, J, E);                             /* add_cur */
            if (walls)
                for (int k = 0; k < n[2]; ++k)
                    for (int j = 0; j < n[1]; ++j) {
                        int64_t cw = cell(n, 0, j, k);
                        E[N + cw] = 0.0;
                        E[2 * N + cw] = 0.0;
                        B[cw] = 0.0;
                    }
        }
    }
    for (int s = 0; xold && disp && s < nspecies; ++s) {
        free(xold[s]);
        free(disp[s]);
    }
    free(xold);
    free(disp);
    free(fp);
    return ok ? 0 : -1;
}

/* ====================================================================== */
/* Adjoint (reverse mode) of one full step, written by hand from the
 * forward routines above.  Differentiation of the step is not in the paper;
 * these routines are the exact vector-Jacobian products of orc_step (the
 * piecewise definitions - floor, the relay point min/max, the CIC weights -
 * are differentiated on the branch the forward value takes).            */

/* Interpolation adjoint at one particle: adds w * lF into the field adjoint
 * lFld of component comp at the 2^D points, and returns dF/dx_d (gradient
 * of the interpolated value with respect to the particle position).      */
static double interp_one(int D, const int n[3], const double *F, int comp, const double *xp,
                         double *lFld, double lval, double grad[3])
{
    int64_t base[3] = {0, 0, 0};
    double w[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < D; ++d) {
        double xi = xp[d] - stagger(comp, d);
        double fl = floor(xi);
        base[d] = (int64_t)fl;
        w[d] = xi - fl;
    }
    double val = 0.0;
    for (int d = 0; d < 3; ++d) grad[d] = 0.0;
    for (int cn = 0; cn < (1 << D); ++cn) {
        int64_t idx[3] = {base[0], base[1], base[2]};
        double wt = 1.0;
        for (int d = 0; d < D; ++d) {
            int bit = (cn >> d) & 1;
            idx[d] += bit;
            wt *= bit ? w[d] : 1.0 - w[d];
        }
        int64_t c = cell(n, idx[0], idx[1], idx[2]);
        val += wt * F[c];
        if (lFld) lFld[c] += wt * lval;
        for (int d = 0; d < D; ++d) {
            double g = (cn >> d) & 1 ? 1.0 : -1.0;   /* d(weight factor)/dx_d */
            for (int e = 0; e < D; ++e)
                if (e != d) g *= ((cn >> e) & 1) ? w[e] : 1.0 - w[e];
            grad[d] += g * F[c];
        }
    }
    return val;
}

/* Boris adjoint: given u^{n-1/2} (u0), fields (Ep, Bp) and the adjoint lu1
 * of u^{n+1/2}, returns the adjoints of u0, Ep, Bp.                       */
static void boris_adjoint(double c, double s, const double u0[3], const double Ep[3], const double Bp[3],
                          const double lu1[3], double lu0[3], double lE[3], double lB[3])
{
    double eps[3], a[3], t[3], w[3], b[3];
    for (int i = 0; i < 3; ++i) {
        eps[i] = 0.5 * s * Ep[i];
        a[i] = c * u0[i] + eps[i];
    }
    double g1 = sqrt(1.0 + (a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) / (c * c));
    double kap = s / (2.0 * c * g1);
    for (int i = 0; i < 3; ++i) t[i] = kap * Bp[i];
    double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double f = 2.0 / (1.0 + tt);
    w[0] = a[0] + (a[1] * t[2] - a[2] * t[1]);
    w[1] = a[1] + (a[2] * t[0] - a[0] * t[2]);
    w[2] = a[2] + (a[0] * t[1] - a[1] * t[0]);
    for (int i = 0; i < 3; ++i) b[i] = f * w[i];
    /* forward: cc = a + b x t + eps, u1 = cc / c */
    double lc[3], la[3], leps[3], lb[3], lt[3], lw[3];
    for (int i = 0; i < 3; ++i) {
        lc[i] = lu1[i] / c;
        la[i] = lc[i];
        leps[i] = lc[i];
    }
    /* b x t: d/db^T lc = t x lc ; d/dt^T lc = lc x b */
    lb[0] = t[1] * lc[2] - t[2] * lc[1];
    lb[1] = t[2] * lc[0] - t[0] * lc[2];
    lb[2] = t[0] * lc[1] - t[1] * lc[0];
    lt[0] = lc[1] * b[2] - lc[2] * b[1];
    lt[1] = lc[2] * b[0] - lc[0] * b[2];
    lt[2] = lc[0] * b[1] - lc[1] * b[0];
    /* b = f w */
    double lf = 0.0;
    for (int i = 0; i < 3; ++i) {
        lw[i] = f * lb[i];
        lf += w[i] * lb[i];
    }
    /* w = a + a x t: d/da^T lw = lw + t x lw ; d/dt^T lw = lw x a */
    la[0] += lw[0] + (t[1] * lw[2] - t[2] * lw[1]);
    la[1] += lw[1] + (t[2] * lw[0] - t[0] * lw[2]);
    la[2] += lw[2] + (t[0] * lw[1] - t[1] * lw[0]);
    lt[0] += lw[1] * a[2] - lw[2] * a[1];
    lt[1] += lw[2] * a[0] - lw[0] * a[2];
    lt[2] += lw[0] * a[1] - lw[1] * a[0];
    /* f = 2/(1+|t|^2): df/dt = -f^2 t */
    for (int i = 0; i < 3; ++i) lt[i] += -lf * f * f * t[i];
    /* t = kap B */
    double lkap = 0.0;
    for (int i = 0; i < 3; ++i) {
        lB[i] = kap * lt[i];
        lkap += Bp[i] * lt[i];
    }
    /* kap = s/(2 c g1): dkap/dg1 = -kap/g1 ; g1 = sqrt(1+|a|^2/c^2) */
    double lg1 = -kap / g1 * lkap;
    for (int i = 0; i < 3; ++i) la[i] += lg1 * a[i] / (c * c * g1);
    /* a = c u0 + eps ; eps = s E / 2 */
    for (int i = 0; i < 3; ++i) {
        lu0[i] = c * la[i];
        leps[i] += la[i];
        lE[i] = 0.5 * s * leps[i];
    }
}

/* One ZigZag segment: values and their derivatives.  For a segment with
 * flux F, weights W, displacement dv (grid dims) in cell i, the value for
 * component m at a corner is F_m * prod_a wf_a (+ F_m sa sb dv_a dv_b / 12
 * with two transverse dims).  dF, dW, ddv hold d/d(input k) for the 2D+ng
 * inputs k.  The adjoint sums lJ(point) * d(value)/d(input k) into lin[k]. */
#define ZZ_NIN 6
static void segment_adjoint(int D, const int n[3], const double *lJ, const double F[3],
                            const double W[3], const double dv[3], const int64_t i[3],
                            double dF[3][ZZ_NIN], double dW[3][ZZ_NIN], double ddv[3][ZZ_NIN], int nin,
                            double *lin)
{
    int64_t N = ncells(n);
    for (int m = 0; m < 3; ++m) {
        int ntrans = 0;
        for (int d = 0; d < D; ++d) ntrans += (d != m);
        for (int cn = 0; cn < (1 << D); ++cn) {
            if (m < D && ((cn >> m) & 1)) continue;
            int64_t idx[3] = {i[0], i[1], i[2]};
            double P = 1.0, C = 1.0;
            for (int d = 0; d < D; ++d) {
                if (d == m) continue;
                int bit = (cn >> d) & 1;
                idx[d] += bit;
                P *= bit ? W[d] : 1.0 - W[d];
                C *= bit ? dv[d] : -dv[d];
            }
            double lam = lJ[m * N + cell(n, idx[0], idx[1], idx[2])];
            double wt = P + (ntrans == 2 ? C / 12.0 : 0.0);
            for (int k = 0; k < nin; ++k) {
                double dP = 0.0, dC = 0.0;
                for (int d = 0; d < D; ++d) {
                    if (d == m) continue;
                    int bit = (cn >> d) & 1;
                    double gP = bit ? dW[d][k] : -dW[d][k];
                    double gC = bit ? ddv[d][k] : -ddv[d][k];
                    double restP = 1.0, restC = 1.0;
                    for (int e = 0; e < D; ++e) {
                        if (e == m || e == d) continue;
                        int be = (cn >> e) & 1;
                        restP *= be ? W[e] : 1.0 - W[e];
                        restC *= be ? dv[e] : -dv[e];
                    }
                    dP += gP * restP;
                    dC += gC * restC;
                }
                double dwt = dP + (ntrans == 2 ? dC / 12.0 : 0.0);
                lin[k] += lam * (dF[m][k] * wt + F[m] * dwt);
            }
        }
    }
}

/* ZigZag adjoint of one particle moving x1 -> x2 with non-grid
 * displacement disp[d >= D]: adds d(sum lJ . J)/d(x1, x2, disp_ng) into
 * lx1[D], lx2[D], ldisp[3].                                             */
static void zigzag_adjoint_one(int D, const int n[3], double q, const double *x1, const double *x2,
                               const double disp[3], const double *lJ, double *lx1, double *lx2,
                               double ldisp[3])
{
    /* inputs: k = d for x1_d, k = D + d for x2_d, k = 2D + (m - D) for disp_m (m >= D) */
    int nin = 2 * D + (3 - D);
    double F1[3], F2[3], W1[3] = {0, 0, 0}, W2[3] = {0, 0, 0}, d1[3] = {0, 0, 0}, d2[3] = {0, 0, 0};
    double dF1[3][ZZ_NIN], dF2[3][ZZ_NIN], dW1[3][ZZ_NIN], dW2[3][ZZ_NIN], dd1[3][ZZ_NIN], dd2[3][ZZ_NIN];
    memset(dF1, 0, sizeof dF1);
    memset(dF2, 0, sizeof dF2);
    memset(dW1, 0, sizeof dW1);
    memset(dW2, 0, sizeof dW2);
    memset(dd1, 0, sizeof dd1);
    memset(dd2, 0, sizeof dd2);
    int64_t i1[3] = {0, 0, 0}, i2[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        if (d < D) {
            double a = x1[d], b = x2[d];
            double fa = floor(a), fb = floor(b);
            double lo = fa < fb ? fa : fb, hi = fa > fb ? fa : fb;
            double mid = 0.5 * (a + b);
            double inner = hi > mid ? hi : mid;
            int mid_used = !(hi > mid);
            double xr = (lo + 1.0) < inner ? (lo + 1.0) : inner;
            if ((lo + 1.0) < inner) mid_used = 0;
            double ra = mid_used ? 0.5 : 0.0, rb = ra;
            int ka = d, kb = D + d;
            F1[d] = q * (xr - a);
            F2[d] = q * (b - xr);
            W1[d] = 0.5 * (a + xr) - fa;
            W2[d] = 0.5 * (b + xr) - fb;
            d1[d] = xr - a;
            d2[d] = b - xr;
            dF1[d][ka] = q * (ra - 1.0);
            dF1[d][kb] = q * rb;
            dF2[d][ka] = -q * ra;
            dF2[d][kb] = q * (1.0 - rb);
            dW1[d][ka] = 0.5 * (1.0 + ra);
            dW1[d][kb] = 0.5 * rb;
            dW2[d][ka] = 0.5 * ra;
            dW2[d][kb] = 0.5 * (1.0 + rb);
            dd1[d][ka] = ra - 1.0;
            dd1[d][kb] = rb;
            dd2[d][ka] = -ra;
            dd2[d][kb] = 1.0 - rb;
            i1[d] = (int64_t)fa;
            i2[d] = (int64_t)fb;
        } else {
            int k = 2 * D + (d - D);
            F1[d] = F2[d] = q * 0.5 * disp[d];
            dF1[d][k] = dF2[d][k] = 0.5 * q;
        }
    }
    double lin[ZZ_NIN] = {0, 0, 0, 0, 0, 0};
    segment_adjoint(D, n, lJ, F1, W1, d1, i1, dF1, dW1, dd1, nin, lin);
    segment_adjoint(D, n, lJ, F2, W2, d2, i2, dF2, dW2, dd2, nin, lin);
    for (int d = 0; d < D; ++d) {
        lx1[d] += lin[d];
        lx2[d] += lin[D + d];
    }
    for (int d = D; d < 3; ++d) ldisp[d] += lin[2 * D + (d - D)];
}

/* Adjoint of orc_step.  The state (x, u, E, B) at the start of the step is
 * read only; on entry lx, lu, lE, lB hold the adjoints of the step's
 * outputs (x^{n+1} before wrapping, u^{n+1/2}, E^{n+1}, B^{n+1/2}); on exit
 * they hold the adjoints of its inputs (x^n, u^{n-1/2}, E^n, B^{n-1/2}).
 * Wrapping x is a shift by a constant and does not change the adjoint.
 * Returns 0, or -1 if scratch could not be allocated.                   */
int orc_step_adjoint(int D, const int n[3], double c, int nspecies, const int64_t *n_per,
                     double **x, double **u, const double *q, const double *sgn,
                     const double *E, const double *B, double **lx, double **lu, double *lE, double *lB)
{
    int64_t N = ncells(n);
    double h = 0.5 * c;
    double *B1 = malloc(sizeof(double) * 3 * (size_t)N);
    double *lJ = malloc(sizeof(double) * 3 * (size_t)N);
    if (!B1 || !lJ) {
        free(B1);
        free(lJ);
        return -1;
    }
    memcpy(B1, B, sizeof(double) * 3 * (size_t)N);
    orc_advance_b(D, n, h, E, B1);                 /* B^n, used by the push */
    /* add_cur: E^{n+1} = ... - J  ->  lJ = -lE */
    for (int64_t k = 0; k < 3 * N; ++k) lJ[k] = -lE[k];
    /* push_e: E^{n+1} = E + c curl- B^{n+1/2}  ->  lB += c curl+ lE */
    orc_advance_b(D, n, -c, lE, lB);
    /* push_half_b2: B^{n+1/2} = B^n - h curl+ E  ->  lE += -h curl- lB */
    orc_advance_e(D, n, -h, lB, lE);
    /* particles (interp_em, push, comp_curr) */
    for (int s = 0; s < nspecies; ++s) {
        int64_t np = n_per[s];
        for (int64_t p = 0; p < np; ++p) {
            double xp[3] = {0, 0, 0}, up[3], Ep[3], Bp[3], g[6][3];
            for (int d = 0; d < D; ++d) xp[d] = x[s][d * np + p];
            for (int i = 0; i < 3; ++i) up[i] = u[s][i * np + p];
            for (int comp = 0; comp < 6; ++comp) {
                double v = interp_one(D, n, comp < 3 ? E + comp * N : B1 + (comp - 3) * N, comp, xp, NULL, 0.0,
                                      g[comp]);
                if (comp < 3) Ep[comp] = v;
                else Bp[comp - 3] = v;
            }
            /* forward push of this particle */
            double u1[3] = {up[0], up[1], up[2]};
            {
                double Ea[3][1], Ba[3][1], uu[3][1];
                for (int i = 0; i < 3; ++i) {
                    Ea[i][0] = Ep[i];
                    Ba[i][0] = Bp[i];
                    uu[i][0] = u1[i];
                }
                orc_boris(1, c, sgn[s], &Ea[0][0], &Ba[0][0], &uu[0][0]);
                for (int i = 0; i < 3; ++i) u1[i] = uu[i][0];
            }
            double gam = sqrt(1.0 + u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
            double disp[3], x2[3] = {0, 0, 0};
            for (int i = 0; i < 3; ++i) disp[i] = c * u1[i] / gam;
            for (int d = 0; d < D; ++d) x2[d] = xp[d] + disp[d];
            /* adjoint of the outputs of this particle */
            double lx2[3] = {0, 0, 0}, lx1[3] = {0, 0, 0}, ldisp[3] = {0, 0, 0}, lu1[3];
            for (int d = 0; d < D; ++d) lx2[d] = lx[s][d * np + p];
            for (int i = 0; i < 3; ++i) lu1[i] = lu[s][i * np + p];
            /* comp_curr */
            zigzag_adjoint_one(D, n, q[s], xp, x2, disp, lJ, lx1, lx2, ldisp);
            /* x2 = x1 + disp (grid dims) */
            for (int d = 0; d < D; ++d) {
                lx1[d] += lx2[d];
                ldisp[d] += lx2[d];
            }
            /* disp = c u1 / gamma(u1) */
            double ul = u1[0] * ldisp[0] + u1[1] * ldisp[1] + u1[2] * ldisp[2];
            for (int i = 0; i < 3; ++i) lu1[i] += c * (ldisp[i] / gam - u1[i] * ul / (gam * gam * gam));
            /* Boris */
            double lu0[3], lEp[3], lBp[3];
            boris_adjoint(c, sgn[s], up, Ep, Bp, lu1, lu0, lEp, lBp);
            /* interpolation: scatter into the field adjoints, gradient in x */
            for (int comp = 0; comp < 6; ++comp) {
                double lval = comp < 3 ? lEp[comp] : lBp[comp - 3];
                double gg[3];
                interp_one(D, n, comp < 3 ? E + comp * N : B1 + (comp - 3) * N, comp, xp,
                           comp < 3 ? lE + comp * N : lB + (comp - 3) * N, lval, gg);
                for (int d = 0; d < D; ++d) lx1[d] += lval * gg[d];
            }
            for (int d = 0; d < D; ++d) lx[s][d * np + p] = lx1[d];
            for (int i = 0; i < 3; ++i) lu[s][i * np + p] = lu0[i];
        }
    }
    /* push_half_b1: B^n = B^{n-1/2} - h curl+ E -> lB unchanged, lE += -h curl- lB */
    orc_advance_e(D, n, -h, lB, lE);
    free(B1);
    free(lJ);
    return 0;
}

/* ====================================================================== */
/* The same step on several host threads, for the CPU baseline: each thread
 * takes a contiguous range of every species' particles through interp_em,
 * push, comp_curr and the wrap with the single-thread routines above (on a
 * private copy of its range) and deposits into a private current array; the
 * field rows stay single-threaded, and the per-thread currents are summed
 * cell by cell in thread order, so a run is reproducible for a given thread
 * count.  Particles and fields equal orc_step's; J (and so E) only differ
 * by the order of the current sums.                                       */

#include <pthread.h>

struct orc_range {
    int D, ns;
    const int *n;
    double c;
    const int64_t *n_per;
    double **x, **u;
    const double *q, *sgn, *E, *B;
    double *J;                 /* this thread's current, 3 N */
    int t, nthreads;
    int ok;
};

static void part_range(int64_t np, int t, int nt, int64_t *a, int64_t *b)
{
    *a = np * t / nt;
    *b = np * (t + 1) / nt;
}

static void *orc_range_worker(void *arg)
{
    struct orc_range *r = (struct orc_range *)arg;
    int D = r->D;
    r->ok = 1;
    for (int s = 0; s < r->ns; ++s) {
        int64_t np = r->n_per[s], a, b;
        part_range(np, r->t, r->nthreads, &a, &b);
        int64_t m = b - a;
        if (m <= 0) continue;
        double *xs = malloc(sizeof(double) * (size_t)(D * m));
        double *xo = malloc(sizeof(double) * (size_t)(D * m));
        double *us = malloc(sizeof(double) * (size_t)(3 * m));
        double *fp = malloc(sizeof(double) * (size_t)(6 * m));
        double *dp = malloc(sizeof(double) * (size_t)(3 * m));
        if (!xs || !xo || !us || !fp || !dp) {
            r->ok = 0;
        } else {
            for (int d = 0; d < D; ++d) memcpy(xs + d * m, r->x[s] + d * np + a, sizeof(double) * (size_t)m);
            for (int i = 0; i < 3; ++i) memcpy(us + i * m, r->u[s] + i * np + a, sizeof(double) * (size_t)m);
            memcpy(xo, xs, sizeof(double) * (size_t)(D * m));
            orc_interp(D, r->n, r->E, r->B, m, xs, fp, fp + 3 * m);
            orc_boris(m, r->c, r->sgn[s], fp, fp + 3 * m, us);
            orc_move(D, m, r->c, us, xs, dp);
            orc_zigzag(D, r->n, r->q[s], m, xo, xs, dp, r->J);
            orc_wrap(D, r->n, m, xs);
            for (int d = 0; d < D; ++d) memcpy(r->x[s] + d * np + a, xs + d * m, sizeof(double) * (size_t)m);
            for (int i = 0; i < 3; ++i) memcpy(r->u[s] + i * np + a, us + i * m, sizeof(double) * (size_t)m);
        }
        free(xs);
        free(xo);
        free(us);
        free(fp);
        free(dp);
        if (!r->ok) break;
    }
    return NULL;
}

struct orc_sum {
    double *J;
    double *const *Jt;
    int64_t a, b;
    int nthreads;
};

static void *orc_sum_worker(void *arg)
{
    struct orc_sum *r = (struct orc_sum *)arg;
    for (int64_t k = r->a; k < r->b; ++k) {
        double acc = 0.0;
        for (int t = 0; t < r->nthreads; ++t) acc += r->Jt[t][k];
        r->J[k] = acc;
    }
    return NULL;
}

/* orc_step on nthreads host threads (Table-1 order as orc_step).  Returns
 * 0, or -1 if memory or threads could not be obtained. */
int orc_step_threads(int D, const int n[3], double c, int nspecies, const int64_t *n_per,
                     double **x, double **u, const double *q, const double *sgn,
                     double *E, double *B, double *J, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    int64_t N = ncells(n);
    double **Jt = calloc((size_t)nthreads, sizeof(double *));
    struct orc_range *rg = calloc((size_t)nthreads, sizeof(struct orc_range));
    struct orc_sum *sm = calloc((size_t)nthreads, sizeof(struct orc_sum));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    int ok = Jt && rg && sm && th;
    for (int t = 0; ok && t < nthreads; ++t) {
        Jt[t] = calloc((size_t)(3 * N), sizeof(double));
        ok = Jt[t] != NULL;
    }
    if (ok) {
        orc_advance_b(D, n, 0.5 * c, E, B);                       /* push_half_b1 */
        for (int t = 0; t < nthreads; ++t) {                       /* interp_em, push, comp_curr */
            struct orc_range r = {D, nspecies, n, c, n_per, x, u, q, sgn, E, B, Jt[t], t, nthreads, 0};
            rg[t] = r;
        }
        int started = 0;
        for (int t = 0; t < nthreads; ++t) {
            if (pthread_create(&th[t], NULL, orc_range_worker, &rg[t]) != 0) break;
            ++started;
        }
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
        ok = started == nthreads;
        for (int t = 0; ok && t < nthreads; ++t) ok = rg[t].ok;
    }
    if (ok) {
        orc_advance_b(D, n, 0.5 * c, E, B);                       /* push_half_b2 */
        orc_advance_e(D, n, c, B, E);                             /* push_e */
        int started = 0;                                           /* J in thread order */
        for (int t = 0; t < nthreads; ++t) {
            sm[t].J = J;
            sm[t].Jt = Jt;
            part_range(3 * N, t, nthreads, &sm[t].a, &sm[t].b);
            sm[t].nthreads = nthreads;
            if (pthread_create(&th[t], NULL, orc_sum_worker, &sm[t]) != 0) break;
            ++started;
        }
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
        ok = started == nthreads;
        if (ok) orc_add_current(n, J, E);                         /* add_cur */
    }
    for (int t = 0; Jt && t < nthreads; ++t) free(Jt[t]);
    free(Jt);
    free(rg);
    free(sm);
    free(th);
    return ok ? 0 : -1;
}
