/*
 * Plain FP64 CPU oracle of the Vlasov-hybrid (VHS) time step.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load this file.  It shares no
 * code, header, table or helper with the GPU library: everything here is
 * written out from the paper (arXiv:1804.03901, Kilian, Schreiner & Spanier)
 * in the most direct form, single-threaded, with no blocking, fusion or
 * reordering beyond what the definitions state.  Build: gcc -O2
 * -ffp-contract=off (no fast-math, no FMA contraction).
 *
 * Grid conventions (Sec. 3.1, Fig. "phasespace"): x in [0, L) is split into
 * nx cells of width dx = L/nx, velocity component d into nv[d] cells of width
 * dv_d = (vmax_d - vmin_d)/nv[d] starting at vmin_d; every gridded value sits
 * at its cell centre, x_i = (i + 1/2) dx, v_j = vmin + (j + 1/2) dv.
 * Phase-space arrays are velocity-major: index ((jz*nvy + jy)*nvx + jx)*nx + i
 * (1D-1V: j*nx + i).  Markers are SoA: x[n], v[vdim*n] (component d at
 * v[d*n + l]), f[n].
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes): corners of a marker's cloud that fall outside the velocity range
 * are dropped without renormalisation; a cell with zero weight sum gets f = 0;
 * the push is kick-then-drift leapfrog with the first kick a full step unless
 * a half first kick is asked for; sinc(y) = sin(y)/y; the Nyquist mode of E is
 * set to zero.
 *
 * Parity of every function here is pinned by the CPU tests (hand sums, closed
 * forms, invariants, the Landau damping root); see tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t vdim;      /* 1 or 3 resolved velocity components */
    int32_t nx;
    int32_t nv[3];
    int32_t pad_;
    double L;
    double vmin[3];
    double vmax[3];
    double dt;
    double q;          /* species charge (normalised: -1 for electrons) */
    double m;          /* species mass */
    double cp;         /* Poisson constant: 4*pi in CGS, 1 in normalised units */
    double B[3];       /* uniform background magnetic field (1D-3V), zero otherwise */
} orc_grid;

static const double ORC_PI = 3.14159265358979323846;

static long n_cells(const orc_grid *g)
{
    long c = g->nx;
    for (int d = 0; d < g->vdim; ++d) c *= g->nv[d];
    return c;
}

static double dv_of(const orc_grid *g, int d)
{
    return (g->vmax[d] - g->vmin[d]) / g->nv[d];
}

/* Cloud-in-cell along one axis (Sec. 2, Fig. "interpolation"): the marker's
 * cloud is one cell wide and centred on the marker, so it overlaps the two
 * cells whose centres bracket it.  Returns the lower of those two cells and the
 * fractional distance `frac` of the marker past that centre: the lower cell
 * gets weight 1-frac, the upper one frac. */
static void cic_axis(double coord, double lo, double h, long *lower, double *frac)
{
    double t = (coord - lo) / h - 0.5;
    double fl = floor(t);
    *lower = (long)fl;
    *frac = t - fl;
}

static long wrap_x(long i, long nx)
{
    long r = i % nx;
    return r < 0 ? r + nx : r;
}

/* ---------------------------------------------------------------------------
 * Reconstruction, Eq. (reconstruction): for every phase cell g,
 *   N_g = sum_l alpha_gl f_l,   D_g = sum_l alpha_gl,   f_g = N_g / D_g,
 * where alpha_gl is the area (volume) overlap of marker l's cloud with cell g
 * divided by the cell area.  In x the domain is periodic; in velocity the
 * overlap with cells outside the grid is simply lost.  Cells that no cloud
 * touches (D_g = 0) get f_g = 0.  Any of Nsum, Dsum, fg may be NULL.
 * ------------------------------------------------------------------------- */
int orc_reconstruct(const orc_grid *g, long n, const double *x, const double *v,
                    const double *f, double *Nsum, double *Dsum, double *fg)
{
    long G = n_cells(g);
    double *Nw = Nsum ? Nsum : (double *)malloc(sizeof(double) * G);
    double *Dw = Dsum ? Dsum : (double *)malloc(sizeof(double) * G);
    if (!Nw || !Dw) return -1;
    memset(Nw, 0, sizeof(double) * G);
    memset(Dw, 0, sizeof(double) * G);
    double dx = g->L / g->nx;
    int ncorner = 1 << (1 + g->vdim);
    for (long l = 0; l < n; ++l) {
        long i0, j0[3];
        double a, b[3];
        cic_axis(x[l], 0.0, dx, &i0, &a);
        for (int d = 0; d < g->vdim; ++d)
            cic_axis(v[(long)d * n + l], g->vmin[d], dv_of(g, d), &j0[d], &b[d]);
        for (int c = 0; c < ncorner; ++c) {
            int up = c & 1;
            double w = up ? a : 1.0 - a;
            long ci = wrap_x(i0 + up, g->nx);
            long idx = 0, stride = g->nx;
            int inside = 1;
            for (int d = 0; d < g->vdim; ++d) {
                int bit = (c >> (1 + d)) & 1;
                long cj = j0[d] + bit;
                if (cj < 0 || cj >= g->nv[d]) { inside = 0; break; }
                w = w * (bit ? b[d] : 1.0 - b[d]);
                idx += cj * stride;
                stride *= g->nv[d];
            }
            if (!inside) continue;
            idx += ci;
            Nw[idx] += w * f[l];
            Dw[idx] += w;
        }
    }
    if (fg)
        for (long k = 0; k < G; ++k) fg[k] = Dw[k] > 0.0 ? Nw[k] / Dw[k] : 0.0;
    if (!Nsum) free(Nw);
    if (!Dsum) free(Dw);
    return 0;
}

/* Paper's contrast case (Sec. 2, the "naive sum"): f_g = sum_l alpha_gl f_l,
 * without normalisation.  Used only by the tests that show the difference. */
int orc_deposit_naive(const orc_grid *g, long n, const double *x, const double *v,
                      const double *f, double *fg)
{
    return orc_reconstruct(g, n, x, v, f, fg, NULL, NULL);
}

/* ---------------------------------------------------------------------------
 * Velocity moments (Sec. 3, algorithm overview; Sec. 3.4, spatial output):
 * midpoint sums over the velocity cells at fixed x cell, no interpolation.
 *   rho_i = q * prod_d dv_d * sum_j f_{i,j}
 *   jx_i  = q * prod_d dv_d * sum_j vx_j f_{i,j}
 *   m2_i  =     prod_d dv_d * sum_j |v_j|^2 f_{i,j}
 * Any output pointer may be NULL.
 * ------------------------------------------------------------------------- */
void orc_moments(const orc_grid *g, const double *fg, double *rho, double *jx, double *m2)
{
    long rows = n_cells(g) / g->nx;
    double vol = 1.0;
    for (int d = 0; d < g->vdim; ++d) vol *= dv_of(g, d);
    for (long i = 0; i < g->nx; ++i) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (long r = 0; r < rows; ++r) {
            long rem = r;
            double vc[3] = {0.0, 0.0, 0.0};
            for (int d = 0; d < g->vdim; ++d) {
                long jd = rem % g->nv[d];
                rem /= g->nv[d];
                vc[d] = g->vmin[d] + (jd + 0.5) * dv_of(g, d);
            }
            double fv = fg[r * g->nx + i];
            s0 += fv;
            s1 += vc[0] * fv;
            s2 += (vc[0] * vc[0] + vc[1] * vc[1] + vc[2] * vc[2]) * fv;
        }
        if (rho) rho[i] = g->q * vol * s0;
        if (jx) jx[i] = g->q * vol * s1;
        if (m2) m2[i] = vol * s2;
    }
}

/* ---------------------------------------------------------------------------
 * Spectral Poisson solve, Eq. (poissonk) with the softening of
 * Eq. (kappasoftening):
 *   rho_hat_m = sum_i rho_i exp(-2 pi i m i / nx)          (plain DFT)
 *   k = 2 pi m' / L,  m' = m for m < nx/2, m - nx above
 *   kappa = k sinc(k dx),  K^2 = k^2 sinc^2(k dx / 2),  sinc(y) = sin(y)/y
 *   E_hat_m = -i cp kappa / K^2 rho_hat_m,   E_hat_0 = 0 (DC removal),
 *   E_hat_{nx/2} = 0 (Nyquist; kappa vanishes there analytically)
 *   E_i = (1/nx) sum_m E_hat_m exp(+2 pi i m i / nx)   (real part)
 * The transform is an O(nx^2) direct sum; twiddle angles use the exact integer
 * reduction (m*i mod nx).  Since E_hat_0 = 0, a constant added to rho cannot
 * change E; the mean of rho is subtracted before the sum, so that a large
 * mean (the charge of the neutralised species) does not leak into the other
 * modes through the rounding of the twiddles.  mode1 (optional) receives
 * (2/nx)|DFT(E)_1|, the amplitude of the longest-wavelength mode of E.
 * ------------------------------------------------------------------------- */
static double sinc(double y) { return y == 0.0 ? 1.0 : sin(y) / y; }

int orc_poisson(int nx, double L, double cp, const double *rho, double *E, double *mode1)
{
    double dx = L / nx;
    double *cs = (double *)malloc(sizeof(double) * nx);
    double *sn = (double *)malloc(sizeof(double) * nx);
    double *er = (double *)malloc(sizeof(double) * nx);
    double *ei = (double *)malloc(sizeof(double) * nx);
    if (!cs || !sn || !er || !ei) return -1;
    for (int r = 0; r < nx; ++r) {
        cs[r] = cos(2.0 * ORC_PI * r / nx);
        sn[r] = sin(2.0 * ORC_PI * r / nx);
    }
    double mean = 0.0;
    for (int i = 0; i < nx; ++i) mean += rho[i];
    mean /= nx;
    for (int m = 0; m < nx; ++m) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < nx; ++i) {
            int r = (int)(((long)m * i) % nx);
            re += (rho[i] - mean) * cs[r];
            im -= (rho[i] - mean) * sn[r];
        }
        if (m == 0 || 2 * m == nx) {
            er[m] = 0.0;
            ei[m] = 0.0;
            continue;
        }
        int mp = (2 * m < nx) ? m : m - nx;
        double k = 2.0 * ORC_PI * mp / L;
        double kappa = k * sinc(k * dx);
        double s = sinc(0.5 * k * dx);
        double K2 = k * k * s * s;
        double c = cp * kappa / K2;
        /* -i * c * (re + i im) = c*im - i*c*re */
        er[m] = c * im;
        ei[m] = -c * re;
    }
    for (int i = 0; i < nx; ++i) {
        double acc = 0.0;
        for (int m = 0; m < nx; ++m) {
            int r = (int)(((long)m * i) % nx);
            acc += er[m] * cs[r] - ei[m] * sn[r];
        }
        E[i] = acc / nx;
    }
    if (mode1) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < nx; ++i) {
            re += E[i] * cs[i % nx];
            im -= E[i] * sn[i % nx];
        }
        *mode1 = 2.0 / nx * sqrt(re * re + im * im);
    }
    free(cs); free(sn); free(er); free(ei);
    return 0;
}

/* Field energy per unit area (Sec. 3.4, thermodynamical output):
 * W = sum_i E_i^2 dx / (2 cp), i.e. 1/(8 pi) sum E^2 dx in CGS. */
double orc_field_energy(int nx, double L, double cp, const double *E)
{
    double s = 0.0;
    for (int i = 0; i < nx; ++i) s += E[i] * E[i];
    return s * (L / nx) / (2.0 * cp);
}

/* Residual charge of the field solve (Sec. 3.4, spatial output): the charge
 * density not accounted for by the field, with the divergence of E taken as
 * a centred difference on the periodic grid and the neutralising background
 * (minus the mean of rho) added to rho:
 *   drho_i = (rho_i - mean(rho)) - (E_{i+1} - E_{i-1}) / (2 dx cp). */
void orc_residual(int nx, double L, double cp, const double *rho, const double *E, double *drho)
{
    double dx = L / nx;
    double mean = 0.0;
    for (int i = 0; i < nx; ++i) mean += rho[i];
    mean /= nx;
    for (int i = 0; i < nx; ++i) {
        int ip = (i + 1) % nx, im = (i + nx - 1) % nx;
        drho[i] = (rho[i] - mean) - (E[ip] - E[im]) / (2.0 * dx * cp);
    }
}

/* Kinetic energy, particle number and coarse-grained entropy from the grid f
 * (Sec. 3.4): Ekin = (m/2) sum |v_j|^2 f dx dV, Ntot = sum f dx dV,
 * S = sum f log f dx dV over cells with f > 0 (sign as printed). */
void orc_energy(const orc_grid *g, const double *fg, double *ekin, double *ntot, double *ent)
{
    long rows = n_cells(g) / g->nx;
    double vol = g->L / g->nx;
    for (int d = 0; d < g->vdim; ++d) vol *= dv_of(g, d);
    double se = 0.0, sn = 0.0, ss = 0.0;
    for (long r = 0; r < rows; ++r) {
        long rem = r;
        double v2 = 0.0;
        for (int d = 0; d < g->vdim; ++d) {
            long jd = rem % g->nv[d];
            rem /= g->nv[d];
            double vc = g->vmin[d] + (jd + 0.5) * dv_of(g, d);
            v2 += vc * vc;
        }
        for (long i = 0; i < g->nx; ++i) {
            double fv = fg[r * g->nx + i];
            se += v2 * fv;
            sn += fv;
            if (fv > 0.0) ss += fv * log(fv);
        }
    }
    if (ekin) *ekin = 0.5 * g->m * se * vol;
    if (ntot) *ntot = sn * vol;
    if (ent) *ent = ss * vol;
}

/* ---------------------------------------------------------------------------
 * Gather and push (Sec. 2, last paragraph of the algorithm description): the
 * field is interpolated to the marker with the same area weighting as the
 * reconstruction, E_l = (1-a) E_{i0} + a E_{i0+1}; then the velocity is
 * advanced with the acceleration (q/m) E_l and the position with the new
 * velocity (kick, then drift), and x is wrapped back into [0, L).  With no
 * magnetic field only the x velocity changes.  `kick` is the fraction of dt
 * used for the velocity update (1, or 1/2 for a half first kick).
 * ------------------------------------------------------------------------- */
void orc_push(const orc_grid *g, long n, double *x, double *v, const double *E, double kick)
{
    double dx = g->L / g->nx;
    double qm = g->q / g->m;
    double tau = g->dt * kick;
    double bmag = sqrt(g->B[0] * g->B[0] + g->B[1] * g->B[1] + g->B[2] * g->B[2]);
    int magnetic = g->vdim == 3 && bmag > 0.0;
    for (long l = 0; l < n; ++l) {
        long i0;
        double a;
        cic_axis(x[l], 0.0, dx, &i0, &a);
        double El = (1.0 - a) * E[wrap_x(i0, g->nx)] + a * E[wrap_x(i0 + 1, g->nx)];
        if (magnetic) {
            /* Boris (1970), the paper's magnetised push: half an electric kick,
             * then the gyration, then the second half kick.  The exact solution
             * of dv/dt = (q/m) v x B over tau turns v about b = B/|B| by the
             * angle -(q/m)|B| tau; the scheme's angle is
             * theta = -2 atan((q/m)|B| tau / 2).  Written here as a rotation
             * (Rodrigues' formula: v cos(theta) + (b x v) sin(theta)
             * + b (b.v)(1 - cos(theta))). */
            double h = 0.5 * qm * El * tau;
            double u[3] = {v[l] + h, v[n + l], v[2 * n + l]};
            double b[3] = {g->B[0] / bmag, g->B[1] / bmag, g->B[2] / bmag};
            double theta = -2.0 * atan(0.5 * qm * bmag * tau);
            double c = cos(theta), s = sin(theta);
            double bu = b[0] * u[0] + b[1] * u[1] + b[2] * u[2];
            double bxu[3] = {b[1] * u[2] - b[2] * u[1], b[2] * u[0] - b[0] * u[2], b[0] * u[1] - b[1] * u[0]};
            double w[3];
            for (int d = 0; d < 3; ++d) w[d] = u[d] * c + bxu[d] * s + b[d] * bu * (1.0 - c);
            v[l] = w[0] + h;
            v[n + l] = w[1];
            v[2 * n + l] = w[2];
        } else {
            v[l] = v[l] + qm * El * tau;
        }
        double xn = x[l] + v[l] * g->dt;
        xn = xn - g->L * floor(xn / g->L);
        if (xn >= g->L) xn -= g->L;
        x[l] = xn;
    }
}

/* ---------------------------------------------------------------------------
 * Step order (Sec. 2, Fig. "algorithm"): after loading, f is reconstructed,
 * rho integrated and E solved (E^0); each step then gathers E^n and pushes,
 * and reconstructs f^{n+1}, rho^{n+1} and E^{n+1}.  diag (2 doubles per step,
 * may be NULL) receives (W, |E_hat_1|) after every step.  E holds E^0 on entry
 * when `have_field` is set, otherwise it is computed first.
 * ------------------------------------------------------------------------- */
int orc_run(const orc_grid *g, long n, double *x, double *v, const double *f,
            int nsteps, int first_kick_half, int have_field, double *E,
            double *diag, double *fg_out, double *D_out, double *rho_out)
{
    long G = n_cells(g);
    double *Nw = (double *)malloc(sizeof(double) * G);
    double *Dw = (double *)malloc(sizeof(double) * G);
    double *fg = (double *)malloc(sizeof(double) * G);
    double *rho = (double *)malloc(sizeof(double) * g->nx);
    if (!Nw || !Dw || !fg || !rho) return -1;
    if (!have_field || nsteps == 0) {
        orc_reconstruct(g, n, x, v, f, Nw, Dw, fg);
        orc_moments(g, fg, rho, NULL, NULL);
        if (!have_field) orc_poisson(g->nx, g->L, g->cp, rho, E, NULL);
    }
    for (int s = 0; s < nsteps; ++s) {
        double kick = (s == 0 && first_kick_half) ? 0.5 : 1.0;
        orc_push(g, n, x, v, E, kick);
        orc_reconstruct(g, n, x, v, f, Nw, Dw, fg);
        orc_moments(g, fg, rho, NULL, NULL);
        double m1 = 0.0;
        orc_poisson(g->nx, g->L, g->cp, rho, E, &m1);
        if (diag) {
            diag[2 * s] = orc_field_energy(g->nx, g->L, g->cp, E);
            diag[2 * s + 1] = m1;
        }
    }
    if (fg_out) memcpy(fg_out, fg, sizeof(double) * G);
    if (D_out) memcpy(D_out, Dw, sizeof(double) * G);
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * g->nx);
    free(Nw); free(Dw); free(fg); free(rho);
    return 0;
}
