/*
 * ssgp_oracle.c -- plain FP64 CPU reference of the split-step Crank-Nicolson
 * (SS-CN) time step for the spin-1 Gross-Pitaevskii equations of
 * arXiv:2009.13507 (Ravisankar, Vudragovic, Muruganandam, Balaz, Adhikari,
 * "Spin-1 spin-orbit- and Rabi-coupled Bose-Einstein condensate solver").
 *
 * TEST INFRASTRUCTURE.  This file is the oracle against which the HIP path
 * is checked.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header, table or helper
 * with the GPU library; it is written to be read against the paper, not to
 * be fast: scalar loops, one sub-step at a time, exactly in the order below.
 *
 * One time step (Sec. 3 "Details about the programs", Table 1, App. A):
 *   1. CALCNU  trap + diagonal density terms (square brackets of Eqs. (1)-(2))
 *              as a pointwise phase (real time) or decay (imaginary time),
 *              all three potentials built from the densities of the input.
 *   2. HERM    off-diagonal c2 terms (curly brackets of Eqs. (1)-(2)) and the
 *              Rabi terms: psi <- exp(-k dt A) psi with the 3x3 Hermitian A of
 *              App. A Eq. (eq:nu), frozen at the input of this sub-step.  The
 *              exponential is evaluated from its power-series definition
 *              (scaling and squaring keeps the argument below 1/8).
 *   3. SO      explicit update psi <- psi - k dt H_SO psi with H_SO the
 *              spin-orbit operator of Sec. 2 (forms after Eq. (3)); the
 *              derivatives are second-order central differences of the input
 *              of this sub-step (App. A Eqs. (p1)-(p2) are the real-time
 *              p_x Sigma_x case).
 *   4. LUX     Crank-Nicolson kinetic step along x on every row/component:
 *              (I + k dt/2 T) psi' = (I - k dt/2 T) psi, T = -1/2 d^2/dx^2 by
 *              the three-point stencil, zero values outside the box.
 *   5. LUY     the same along y (2D only).
 *   6. RENORM  (imaginary time only) psi_j <- d_j psi_j with d_j from
 *              App. A Eq. (DJ) (fixed magnetisation) or Eq. (DJ2) (norm only).
 * k = i in real time and k = 1 in imaginary time (Delta -> -i Delta).
 *
 * Readings where the paper is silent (each listed with its reason in the
 * design notes of the repository): Lie splitting with full steps in the order
 * above; Omega~ = Omega/sqrt(2); Dirichlet zero ghosts; rectangle-rule
 * integrals; grid x_i = -nx dx/2 + i dx; rms sizes normalised per component.
 *
 * Layout: psi[(j*ny + iy)*nx + ix], j = 0,1,2 for spin components +1, 0, -1,
 * x fastest.  In 1D ny = 1 and dy is ignored (area element dx).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    int dim, nx, ny;
    double dx, dy;
    double c0, c2, gamma, omega, kappa;
    double dt;
    int imag;      /* 1: imaginary time, 0: real time (OPT_PROP of Table 2) */
    int so;        /* spin-orbit form, see enum below (OPT_SO of Table 2)   */
    int renorm;    /* 0 auto, 1 norm only (DJ2), 2 fixed m (DJ)             */
    double mag0;   /* m of Eq. (noma), used by DJ                           */
} ora_cfg;

enum { SO_NONE = 0, SO_PX_SX = 1, SO_PX_SY = 2, SO_PX_SZ = 3,
       SO_RASHBA = 4, SO_DRESSELHAUS = 5, SO_ERD = 6 };
enum { RN_AUTO = 0, RN_NORM = 1, RN_FIXED_M = 2 };

static size_t npts(const ora_cfg *c) { return (size_t)c->nx * (size_t)(c->dim == 2 ? c->ny : 1); }
static int nrows(const ora_cfg *c) { return c->dim == 2 ? c->ny : 1; }
static double xc(const ora_cfg *c, int i) { return -0.5 * c->nx * c->dx + i * c->dx; }
static double yc(const ora_cfg *c, int i) { return c->dim == 2 ? -0.5 * c->ny * c->dy + i * c->dy : 0.0; }
static double darea(const ora_cfg *c) { return c->dim == 2 ? c->dx * c->dy : c->dx; }
/* k of the header: i for real time, 1 for imaginary time */
static cplx kfac(const ora_cfg *c) { return c->imag ? 1.0 : I; }

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the parallel loops that follow (for timing; the steps and the
 * norms do not depend on it, the adjoint's Omega derivative only through the
 * order of its sum) */
void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------- CALCNU */
/* Diagonal part of Eqs. (1)-(2): phi_{+-1} = V + c0 rho + c2 (rho_{+-1} - rho_{-+1} + rho_0),
 * phi_0 = V + c0 rho + c2 (rho_{+1} + rho_{-1}), V = (x^2 + kappa^2 y^2)/2 (Sec. 2). */
void ora_calcnu(const ora_cfg *c, cplx *psi)
{
    size_t np = npts(c);
    cplx k = kfac(c);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)np; p++) {
        int ix = (int)(p % c->nx), iy = (int)(p / c->nx);
        double x = xc(c, ix), y = yc(c, iy);
        double V = 0.5 * (x * x + c->kappa * c->kappa * y * y);
        cplx *up = psi + p, *u0 = psi + np + p, *um = psi + 2 * np + p;
        double rp = creal(*up) * creal(*up) + cimag(*up) * cimag(*up);
        double r0 = creal(*u0) * creal(*u0) + cimag(*u0) * cimag(*u0);
        double rm = creal(*um) * creal(*um) + cimag(*um) * cimag(*um);
        double rho = rp + r0 + rm;
        double php = V + c->c0 * rho + c->c2 * (rp - rm + r0);
        double ph0 = V + c->c0 * rho + c->c2 * (rp + rm);
        double phm = V + c->c0 * rho + c->c2 * (rm - rp + r0);
        *up *= cexp(-k * c->dt * php);
        *u0 *= cexp(-k * c->dt * ph0);
        *um *= cexp(-k * c->dt * phm);
    }
}

/* ------------------------------------------------------------------ HERM */
/* A = [[0, a, 0], [a*, 0, b], [0, b*, 0]], a = c2 psi_{-1}^* psi_0 + Omega~,
 * b = c2 psi_0^* psi_{+1} + Omega~ (App. A, Eq. (eq:nu)); Omega~ = Omega/sqrt 2.
 * exp(z A) v = sum_n (z A)^n v / n!, with z A scaled by 2^-s so that its
 * row-sum norm is at most 1/8 and the series cut after 20 terms (remainder
 * below 1e-30 relative), then applied 2^s times. */
static void herm_point(cplx a, cplx b, cplx z, cplx v[3])
{
    double na = cabs(a), nb = cabs(b);
    double nrm = cabs(z) * (na + nb);
    int s = 0;
    while (nrm > 0.125) { nrm *= 0.5; s++; }
    cplx zs = z * ldexp(1.0, -s);
    for (int rep = 0; rep < (1 << s); rep++) {
        cplx sum[3] = { v[0], v[1], v[2] }, t[3] = { v[0], v[1], v[2] };
        for (int n = 1; n <= 20; n++) {
            cplx At0 = a * t[1];
            cplx At1 = conj(a) * t[0] + b * t[2];
            cplx At2 = conj(b) * t[1];
            t[0] = zs * At0 / n; t[1] = zs * At1 / n; t[2] = zs * At2 / n;
            sum[0] += t[0]; sum[1] += t[1]; sum[2] += t[2];
        }
        v[0] = sum[0]; v[1] = sum[1]; v[2] = sum[2];
    }
}

void ora_herm(const ora_cfg *c, cplx *psi)
{
    size_t np = npts(c);
    cplx z = -kfac(c) * c->dt;
    double om = c->omega / sqrt(2.0);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)np; p++) {
        cplx v[3] = { psi[p], psi[np + p], psi[2 * np + p] };
        cplx a = c->c2 * conj(v[2]) * v[1] + om;
        cplx b = c->c2 * conj(v[1]) * v[0] + om;
        herm_point(a, b, z, v);
        psi[p] = v[0]; psi[np + p] = v[1]; psi[2 * np + p] = v[2];
    }
}

/* -------------------------------------------------------------------- SO */
/* central differences with zero values outside the box */
static cplx ddx(const ora_cfg *c, const cplx *f, int ix, int iy)
{
    cplx fp = ix + 1 < c->nx ? f[(size_t)iy * c->nx + ix + 1] : 0.0;
    cplx fm = ix - 1 >= 0 ? f[(size_t)iy * c->nx + ix - 1] : 0.0;
    return (fp - fm) / (2.0 * c->dx);
}
static cplx ddy(const ora_cfg *c, const cplx *f, int ix, int iy)
{
    if (c->dim != 2) return 0.0;
    cplx fp = iy + 1 < c->ny ? f[(size_t)(iy + 1) * c->nx + ix] : 0.0;
    cplx fm = iy - 1 >= 0 ? f[(size_t)(iy - 1) * c->nx + ix] : 0.0;
    return (fp - fm) / (2.0 * c->dy);
}

/* out = H_SO psi, with p = -i d/dx, gamma~ = gamma/sqrt 2 and the spin-1
 * matrices of Eq. (3):
 *  p_x Sigma_x : (H psi)_{+-1} = -i g~ d_x psi_0,  (H psi)_0 = -i g~ d_x (psi_{+1} + psi_{-1})
 *  p_x Sigma_y : (H psi)_{+-1} = -+ g~ d_x psi_0,  (H psi)_0 = g~ d_x (psi_{+1} - psi_{-1})
 *                (derived from Sigma_y of Eq. (3); the printed forms carry an
 *                extra factor -i that would make the operator non-Hermitian)
 *  p_x Sigma_z : (H psi)_{+-1} = -+ i g d_x psi_{+-1},  (H psi)_0 = 0
 *  2D g(eta p_y Sigma_x - p_x Sigma_y), eta = 1 (Rashba), -1 (Dresselhaus), 0:
 *    (H psi)_{+-1} = -i g~ [eta d_y psi_0 +- i d_x psi_0]
 *    (H psi)_0     = -i g~ [-i d_x psi_{+1} + i d_x psi_{-1} + eta d_y (psi_{+1} + psi_{-1})]
 */
void ora_apply_hso(const ora_cfg *c, const cplx *psi, cplx *out)
{
    size_t np = npts(c);
    const cplx *fp = psi, *f0 = psi + np, *fm = psi + 2 * np;
    double g = c->gamma, gt = c->gamma / sqrt(2.0);
    double eta = c->so == SO_RASHBA ? 1.0 : (c->so == SO_DRESSELHAUS ? -1.0 : 0.0);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)np; p++) {
        int ix = (int)(p % c->nx), iy = (int)(p / c->nx);
        cplx hp = 0, h0 = 0, hm = 0;
        switch (c->so) {
        case SO_PX_SX:
            hp = -I * gt * ddx(c, f0, ix, iy);
            hm = hp;
            h0 = -I * gt * (ddx(c, fp, ix, iy) + ddx(c, fm, ix, iy));
            break;
        case SO_PX_SY:
            hp = -gt * ddx(c, f0, ix, iy);
            hm = gt * ddx(c, f0, ix, iy);
            h0 = gt * (ddx(c, fp, ix, iy) - ddx(c, fm, ix, iy));
            break;
        case SO_PX_SZ:
            hp = -I * g * ddx(c, fp, ix, iy);
            hm = I * g * ddx(c, fm, ix, iy);
            h0 = 0;
            break;
        case SO_RASHBA: case SO_DRESSELHAUS: case SO_ERD:
            hp = -I * gt * (eta * ddy(c, f0, ix, iy) + I * ddx(c, f0, ix, iy));
            hm = -I * gt * (eta * ddy(c, f0, ix, iy) - I * ddx(c, f0, ix, iy));
            h0 = -I * gt * (-I * ddx(c, fp, ix, iy) + I * ddx(c, fm, ix, iy)
                            + eta * (ddy(c, fp, ix, iy) + ddy(c, fm, ix, iy)));
            break;
        default:
            break;
        }
        out[p] = hp; out[np + p] = h0; out[2 * np + p] = hm;
    }
}

/* psi <- psi - k dt H_SO psi, every derivative taken from the input (App. A) */
void ora_so(const ora_cfg *c, cplx *psi)
{
    if (c->so == SO_NONE) return;
    size_t np = npts(c);
    cplx *h = malloc(3 * np * sizeof(cplx));
    ora_apply_hso(c, psi, h);
    cplx kd = kfac(c) * c->dt;
    for (size_t q = 0; q < 3 * np; q++) psi[q] -= kd * h[q];
    free(h);
}

/* ------------------------------------------------------------ LUX / LUY */
/* Thomas elimination of tridiag(o, d, o) x = r along one strided line, no
 * pivoting (the matrices here are diagonally dominant). r is overwritten. */
static void thomas(int n, cplx d, cplx o, cplx *r, size_t stride, cplx *cp)
{
    cp[0] = o / d;
    r[0] = r[0] / d;
    for (int i = 1; i < n; i++) {
        cplx m = d - o * cp[i - 1];
        cp[i] = o / m;
        r[(size_t)i * stride] = (r[(size_t)i * stride] - o * r[(size_t)(i - 1) * stride]) / m;
    }
    for (int i = n - 2; i >= 0; i--)
        r[(size_t)i * stride] -= cp[i] * r[(size_t)(i + 1) * stride];
}

/* One line: rhs = (I - s T) f, then solve (I + s T) f' = rhs, with
 * T = tridiag(-1/(2h^2), 1/h^2, -1/(2h^2)) and s the complex factor given.
 * With conj_adjoint set, applies instead the adjoint (I - s T)^H (I + s T)^-H. */
static void cn_line(int n, double h, cplx s, cplx *f, size_t stride, cplx *work, int adjoint)
{
    cplx *rhs = work, *cp = work + n;
    double tdiag = 1.0 / (h * h), toff = -0.5 / (h * h);
    if (!adjoint) {
        for (int i = 0; i < n; i++) {
            cplx fl = i > 0 ? f[(size_t)(i - 1) * stride] : 0.0;
            cplx fr = i + 1 < n ? f[(size_t)(i + 1) * stride] : 0.0;
            cplx fi = f[(size_t)i * stride];
            rhs[i] = fi - s * (tdiag * fi + toff * (fl + fr));
        }
        thomas(n, 1.0 + s * tdiag, s * toff, rhs, 1, cp);
    } else {
        /* forward map M = A^-1 B with A = I + sT, B = I - sT; M^H = B^H A^-H */
        for (int i = 0; i < n; i++) rhs[i] = f[(size_t)i * stride];
        thomas(n, conj(1.0 + s * tdiag), conj(s * toff), rhs, 1, cp);
        for (int i = 0; i < n; i++) {
            cplx fl = i > 0 ? rhs[i - 1] : 0.0;
            cplx fr = i + 1 < n ? rhs[i + 1] : 0.0;
            f[(size_t)i * stride] = rhs[i] - conj(s) * (tdiag * rhs[i] + toff * (fl + fr));
        }
        return;
    }
    for (int i = 0; i < n; i++) f[(size_t)i * stride] = rhs[i];
}

static void cn_x_impl(const ora_cfg *c, cplx *psi, int adjoint)
{
    int ny = nrows(c);
    cplx s = 0.5 * kfac(c) * c->dt;
#pragma omp parallel
    {
        cplx *work = malloc(2 * (size_t)c->nx * sizeof(cplx));
#pragma omp for schedule(static)
        for (long line = 0; line < 3L * ny; line++)
            cn_line(c->nx, c->dx, s, psi + (size_t)line * c->nx, 1, work, adjoint);
        free(work);
    }
}

static void cn_y_impl(const ora_cfg *c, cplx *psi, int adjoint)
{
    if (c->dim != 2) return;
    size_t np = npts(c);
    cplx s = 0.5 * kfac(c) * c->dt;
#pragma omp parallel
    {
        cplx *work = malloc(2 * (size_t)c->ny * sizeof(cplx));
#pragma omp for schedule(static)
        for (long line = 0; line < 3L * c->nx; line++) {
            int j = (int)(line / c->nx), ix = (int)(line % c->nx);
            cn_line(c->ny, c->dy, s, psi + j * np + ix, (size_t)c->nx, work, adjoint);
        }
        free(work);
    }
}

void ora_cn_x(const ora_cfg *c, cplx *psi) { cn_x_impl(c, psi, 0); }
void ora_cn_y(const ora_cfg *c, cplx *psi) { cn_y_impl(c, psi, 0); }

/* ---------------------------------------------------------------- RENORM */
/* N_j = dA sum |psi_j|^2 (rectangle rule), summed in index order */
void ora_norms(const ora_cfg *c, const cplx *psi, double N[3])
{
    size_t np = npts(c);
    for (int j = 0; j < 3; j++) {
        double s = 0.0;
        for (size_t p = 0; p < np; p++) {
            cplx v = psi[j * np + p];
            s += creal(v) * creal(v) + cimag(v) * cimag(v);
        }
        N[j] = s * darea(c);
    }
}

/* Which rescaling applies: Eq. (DJ) keeps m fixed and is used only when the
 * Hamiltonian conserves magnetisation (no Rabi term and no spin-orbit term
 * that fails to commute with Sigma_z); otherwise Eq. (DJ2). */
int ora_uses_fixed_m(const ora_cfg *c)
{
    if (c->renorm == RN_NORM) return 0;
    if (c->renorm == RN_FIXED_M) return 1;
    int so_commutes = c->so == SO_NONE || c->so == SO_PX_SZ || c->gamma == 0.0;
    return c->omega == 0.0 && so_commutes;
}

/* d_j of Eq. (DJ) or Eq. (DJ2).  Returns 1 when Eq. (DJ) could not be used
 * (|m| >= 1, an empty +-1 component or a negative radicand) and Eq. (DJ2)
 * was applied instead. */
int ora_renorm_factors(const ora_cfg *c, const double N[3], double d[3])
{
    double Np = N[0], N0 = N[1], Nm = N[2];
    if (ora_uses_fixed_m(c)) {
        double m = c->mag0;
        if (fabs(m) < 1.0 && Np > 0.0 && Nm > 0.0) {
            double d0 = sqrt(1.0 - m * m) / sqrt(N0 + sqrt(4.0 * (1.0 - m * m) * Np * Nm + m * m * N0 * N0));
            double rp = 1.0 + m - d0 * d0 * N0, rm = 1.0 - m - d0 * d0 * N0;
            if (rp >= 0.0 && rm >= 0.0) {
                d[0] = sqrt(rp) / sqrt(2.0 * Np);
                d[1] = d0;
                d[2] = sqrt(rm) / sqrt(2.0 * Nm);
                return 0;
            }
        }
        double dd = 1.0 / sqrt(N0 + Np + Nm);
        d[0] = d[1] = d[2] = dd;
        return 1;
    }
    double dd = 1.0 / sqrt(N0 + Np + Nm);
    d[0] = d[1] = d[2] = dd;
    return 0;
}

int ora_renorm(const ora_cfg *c, cplx *psi)
{
    size_t np = npts(c);
    double N[3], d[3];
    ora_norms(c, psi, N);
    int fb = ora_renorm_factors(c, N, d);
    for (int j = 0; j < 3; j++)
        for (size_t p = 0; p < np; p++) psi[j * np + p] *= d[j];
    return fb;
}

/* ------------------------------------------------------------------ step */
void ora_step(const ora_cfg *c, cplx *psi, long nsteps)
{
    for (long s = 0; s < nsteps; s++) {
        ora_calcnu(c, psi);
        ora_herm(c, psi);
        ora_so(c, psi);
        ora_cn_x(c, psi);
        ora_cn_y(c, psi);
        if (c->imag) ora_renorm(c, psi);
    }
}

/* ------------------------------------------- second-order pointwise stage */
/* Opt-in second-order (Strang) scheme, beyond the paper.  The pointwise part
 * of Eqs. (1)-(2) (trap and density terms, c2 and Rabi couplings) is the flow
 * psi' = -k (Phi(psi) + A(psi)) psi at every point, Phi = diag(phi_j) of
 * CALCNU and A the matrix of HERM (App. A, Eq. (eq:nu)).  CALCNU and HERM
 * take Phi and A frozen at their input, which is first order in the step for
 * c2 != 0.  This stage integrates the flow over tau by the exponential
 * midpoint rule:
 *   1. predictor: psi_m = HERM(tau/2) CALCNU(tau/2) psi (the paper's two
 *      sub-steps over half the interval);
 *   2. Phi_m = Phi(psi_m), A_m = A(psi_m);
 *   3. psi <- exp(-k tau/2 Phi_m) exp(-k tau A_m) exp(-k tau/2 Phi_m) psi,
 *      the symmetric product of the two frozen exponentials.
 * psi_m is within O(tau^2) of the exact midpoint value, so the stage has a
 * local error O(tau^3).  The exponentials are those of CALCNU (the exp of
 * each diagonal entry) and HERM (the power series of exp(z A_m) above). */
static void phi_point(const ora_cfg *c, double V, const cplx v[3], double phi[3])
{
    double rp = creal(v[0]) * creal(v[0]) + cimag(v[0]) * cimag(v[0]);
    double r0 = creal(v[1]) * creal(v[1]) + cimag(v[1]) * cimag(v[1]);
    double rm = creal(v[2]) * creal(v[2]) + cimag(v[2]) * cimag(v[2]);
    double rho = rp + r0 + rm;
    phi[0] = V + c->c0 * rho + c->c2 * (rp - rm + r0);
    phi[1] = V + c->c0 * rho + c->c2 * (rp + rm);
    phi[2] = V + c->c0 * rho + c->c2 * (rm - rp + r0);
}

static void ab_point(const ora_cfg *c, const cplx v[3], cplx *a, cplx *b)
{
    double om = c->omega / sqrt(2.0);
    *a = c->c2 * conj(v[2]) * v[1] + om;
    *b = c->c2 * conj(v[1]) * v[0] + om;
}

void ora_pointwise2(const ora_cfg *c, cplx *psi, double tau)
{
    size_t np = npts(c);
    cplx k = kfac(c);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)np; p++) {
        int ix = (int)(p % c->nx), iy = (int)(p / c->nx);
        double x = xc(c, ix), y = yc(c, iy);
        double V = 0.5 * (x * x + c->kappa * c->kappa * y * y);
        cplx v[3] = { psi[p], psi[np + p], psi[2 * np + p] };
        /* 1. predictor over tau/2 */
        cplx m[3] = { v[0], v[1], v[2] };
        double phi[3];
        cplx a, b;
        phi_point(c, V, m, phi);
        for (int j = 0; j < 3; j++) m[j] *= cexp(-k * (0.5 * tau) * phi[j]);
        ab_point(c, m, &a, &b);
        herm_point(a, b, -k * (0.5 * tau), m);
        /* 2. coefficients at the midpoint */
        phi_point(c, V, m, phi);
        ab_point(c, m, &a, &b);
        /* 3. symmetric product of the frozen exponentials */
        for (int j = 0; j < 3; j++) v[j] *= cexp(-k * (0.5 * tau) * phi[j]);
        herm_point(a, b, -k * tau, v);
        for (int j = 0; j < 3; j++) v[j] *= cexp(-k * (0.5 * tau) * phi[j]);
        psi[p] = v[0]; psi[np + p] = v[1]; psi[2 * np + p] = v[2];
    }
}

/* ----------------------------------------------------------- observables */
/* out[0..15] = N+1, N0, N-1, N, M, E, E_kin, E_trap, E_c0, E_c2, E_rabi, E_so,
 *              rms+1, rms0, rms-1, rms_total.
 * Eq. (5) on the grid: the gradient term is the forward difference over every
 * link including the two links to the zero ghosts of each line (so it equals
 * <psi, T psi> of the stepped Laplacian); the spin-orbit term is
 * Re sum_j psi_j^* (H_SO psi)_j with the same H_SO as the SO sub-step. */
void ora_observables(const ora_cfg *c, const cplx *psi, double *out)
{
    size_t np = npts(c);
    int ny = nrows(c);
    double dA = darea(c);
    double om = c->omega / sqrt(2.0);
    cplx *h = calloc(3 * np, sizeof(cplx));
    ora_apply_hso(c, psi, h);
    double N[3] = { 0, 0, 0 }, ekin = 0, etrap = 0, ec0 = 0, ec2 = 0, erabi = 0, eso = 0;
    double r2w[3] = { 0, 0, 0 };
    for (int iy = 0; iy < ny; iy++) {
        for (int ix = 0; ix < c->nx; ix++) {
            size_t p = (size_t)iy * c->nx + ix;
            double x = xc(c, ix), y = yc(c, iy);
            double V = 0.5 * (x * x + c->kappa * c->kappa * y * y);
            double r2 = x * x + y * y;
            cplx up = psi[p], u0 = psi[np + p], um = psi[2 * np + p];
            double rj[3];
            for (int j = 0; j < 3; j++) {
                cplx v = psi[j * np + p];
                rj[j] = creal(v) * creal(v) + cimag(v) * cimag(v);
                N[j] += rj[j];
                r2w[j] += r2 * rj[j];
                /* links to the right / above, and the link from the left / below ghost */
                cplx vr = ix + 1 < c->nx ? psi[j * np + p + 1] : 0.0;
                double gx = cabs(vr - v);
                ekin += 0.5 * gx * gx / (c->dx * c->dx);
                if (ix == 0) ekin += 0.5 * cabs(v) * cabs(v) / (c->dx * c->dx);
                if (c->dim == 2) {
                    cplx vu = iy + 1 < c->ny ? psi[j * np + p + c->nx] : 0.0;
                    double gy = cabs(vu - v);
                    ekin += 0.5 * gy * gy / (c->dy * c->dy);
                    if (iy == 0) ekin += 0.5 * cabs(v) * cabs(v) / (c->dy * c->dy);
                }
                eso += creal(conj(v) * h[j * np + p]);
            }
            double rho = rj[0] + rj[1] + rj[2];
            etrap += V * rho;
            ec0 += 0.5 * c->c0 * rho * rho;
            ec2 += 0.5 * c->c2 * (rj[0] * rj[0] + rj[2] * rj[2] + 2.0 * rj[0] * rj[1]
                                  + 2.0 * rj[2] * rj[1] - 2.0 * rj[0] * rj[2]
                                  + 4.0 * creal(conj(um) * u0 * u0 * conj(up)));
            erabi += 2.0 * om * creal((conj(up) + conj(um)) * u0);
        }
    }
    free(h);
    for (int j = 0; j < 3; j++) out[j] = N[j] * dA;
    out[3] = out[0] + out[1] + out[2];
    out[4] = out[0] - out[2];
    out[6] = ekin * dA; out[7] = etrap * dA; out[8] = ec0 * dA; out[9] = ec2 * dA;
    out[10] = erabi * dA; out[11] = eso * dA;
    out[5] = out[6] + out[7] + out[8] + out[9] + out[10] + out[11];
    for (int j = 0; j < 3; j++) out[12 + j] = N[j] > 0.0 ? sqrt(r2w[j] / N[j]) : 0.0;
    double ntot = N[0] + N[1] + N[2];
    out[15] = ntot > 0.0 ? sqrt((r2w[0] + r2w[1] + r2w[2]) / ntot) : 0.0;
}

/* ---------------------------------------------------------- adjoint step */
/* Reverse-mode derivative of one real-time step, in the gradient convention
 * g = dL/dRe(psi) + i dL/dIm(psi).  The linear sub-steps take their adjoints
 * from the definitions (CN: M = A^-1 B -> M^H = B^H A^-H; SO: I - i dt H ->
 * I + i dt H).  The pointwise map P = HERM o CALCNU is differentiated by
 * forward-mode dual numbers: 6 real tangent directions (Re, Im of the three
 * components) plus Omega, giving the real 6x6 Jacobian J_R and dP/dOmega at
 * each point; the pull-back is J_R^T g. */
#define NT 7
typedef struct { cplx v; cplx d[NT]; } dual;

static dual dl_const(cplx v) { dual r; r.v = v; for (int k = 0; k < NT; k++) r.d[k] = 0; return r; }
static dual dl_add(dual a, dual b) { dual r; r.v = a.v + b.v; for (int k = 0; k < NT; k++) r.d[k] = a.d[k] + b.d[k]; return r; }
static dual dl_mul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int k = 0; k < NT; k++) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
static dual dl_scale(dual a, cplx s) { dual r; r.v = a.v * s; for (int k = 0; k < NT; k++) r.d[k] = a.d[k] * s; return r; }
static dual dl_conj(dual a) { dual r; r.v = conj(a.v); for (int k = 0; k < NT; k++) r.d[k] = conj(a.d[k]); return r; }
static dual dl_exp(dual a) { dual r; r.v = cexp(a.v); for (int k = 0; k < NT; k++) r.d[k] = r.v * a.d[k]; return r; }
static dual dl_abs2(dual a) { return dl_mul(a, dl_conj(a)); }

static void pointwise_dual(const ora_cfg *c, double V, cplx om_val, dual v[3])
{
    cplx k = kfac(c);
    /* CALCNU */
    dual rp = dl_abs2(v[0]), r0 = dl_abs2(v[1]), rm = dl_abs2(v[2]);
    dual rho = dl_add(dl_add(rp, r0), rm);
    dual base = dl_add(dl_const(V), dl_scale(rho, c->c0));
    dual php = dl_add(base, dl_scale(dl_add(dl_add(rp, dl_scale(rm, -1.0)), r0), c->c2));
    dual ph0 = dl_add(base, dl_scale(dl_add(rp, rm), c->c2));
    dual phm = dl_add(base, dl_scale(dl_add(dl_add(rm, dl_scale(rp, -1.0)), r0), c->c2));
    v[0] = dl_mul(v[0], dl_exp(dl_scale(php, -k * c->dt)));
    v[1] = dl_mul(v[1], dl_exp(dl_scale(ph0, -k * c->dt)));
    v[2] = dl_mul(v[2], dl_exp(dl_scale(phm, -k * c->dt)));
    /* HERM: Omega~ carries the 7th tangent direction */
    dual omt = dl_const(om_val / sqrt(2.0));
    omt.d[6] = 1.0 / sqrt(2.0);
    dual a = dl_add(dl_scale(dl_mul(dl_conj(v[2]), v[1]), c->c2), omt);
    dual b = dl_add(dl_scale(dl_mul(dl_conj(v[1]), v[0]), c->c2), omt);
    cplx z = -k * c->dt;
    double nrm = cabs(z) * (cabs(a.v) + cabs(b.v));
    int s = 0;
    while (nrm > 0.125) { nrm *= 0.5; s++; }
    cplx zs = z * ldexp(1.0, -s);
    for (int rep = 0; rep < (1 << s); rep++) {
        dual sum[3] = { v[0], v[1], v[2] }, t[3] = { v[0], v[1], v[2] };
        for (int n = 1; n <= 20; n++) {
            dual At0 = dl_mul(a, t[1]);
            dual At1 = dl_add(dl_mul(dl_conj(a), t[0]), dl_mul(b, t[2]));
            dual At2 = dl_mul(dl_conj(b), t[1]);
            t[0] = dl_scale(At0, zs / n); t[1] = dl_scale(At1, zs / n); t[2] = dl_scale(At2, zs / n);
            for (int j = 0; j < 3; j++) sum[j] = dl_add(sum[j], t[j]);
        }
        for (int j = 0; j < 3; j++) v[j] = sum[j];
    }
}

/* Value of P = HERM o CALCNU alone, through the dual-number code (lets the
 * tests check that the differentiated map is the stepped map). */
void ora_pointwise_dual_value(const ora_cfg *c, cplx *psi)
{
    size_t np = npts(c);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)np; p++) {
        int ix = (int)(p % c->nx), iy = (int)(p / c->nx);
        double x = xc(c, ix), y = yc(c, iy);
        double V = 0.5 * (x * x + c->kappa * c->kappa * y * y);
        dual v[3];
        for (int j = 0; j < 3; j++) v[j] = dl_const(psi[j * np + p]);
        pointwise_dual(c, V, c->omega, v);
        for (int j = 0; j < 3; j++) psi[j * np + p] = v[j].v;
    }
}

/* lambda: on entry dL/dpsi^{n+1}, on exit dL/dpsi^n.  psi_n: the step input.
 * *dL_domega is incremented by the derivative of L with respect to the Omega
 * of this step.  Real time only. */
int ora_step_adjoint(const ora_cfg *c, const cplx *psi_n, cplx *lam, double *dL_domega)
{
    if (c->imag) return -1;
    size_t np = npts(c);
    cn_y_impl(c, lam, 1);
    cn_x_impl(c, lam, 1);
    if (c->so != SO_NONE) {
        cplx *h = malloc(3 * np * sizeof(cplx));
        ora_apply_hso(c, lam, h);
        /* S = I - k dt H  ->  S^H = I - conj(k) dt H (H Hermitian) */
        cplx kd = conj(kfac(c)) * c->dt;
        for (size_t q = 0; q < 3 * np; q++) lam[q] -= kd * h[q];
        free(h);
    }
    double domega = 0.0;
#pragma omp parallel for schedule(static) reduction(+:domega)
    for (long p = 0; p < (long)np; p++) {
        int ix = (int)(p % c->nx), iy = (int)(p / c->nx);
        double x = xc(c, ix), y = yc(c, iy);
        double V = 0.5 * (x * x + c->kappa * c->kappa * y * y);
        dual v[3];
        for (int j = 0; j < 3; j++) {
            v[j] = dl_const(psi_n[j * np + p]);
            v[j].d[2 * j] = 1.0;       /* d/dRe psi_j */
            v[j].d[2 * j + 1] = I;     /* d/dIm psi_j */
        }
        pointwise_dual(c, V, c->omega, v);
        cplx g[3] = { lam[p], lam[np + p], lam[2 * np + p] };
        /* (J_R^T g)_k = sum_j Re(conj(g_j) dy_j/dt_k) */
        double gin[6];
        for (int k = 0; k < 6; k++) {
            double s = 0.0;
            for (int j = 0; j < 3; j++) s += creal(conj(g[j]) * v[j].d[k]);
            gin[k] = s;
        }
        double dom = 0.0;
        for (int j = 0; j < 3; j++) dom += creal(conj(g[j]) * v[j].d[6]);
        domega += dom;
        for (int j = 0; j < 3; j++) lam[j * np + p] = gin[2 * j] + I * gin[2 * j + 1];
    }
    *dL_domega += domega;
    return 0;
}

/* adjoint sub-steps exposed for the dot-product tests */
void ora_cn_x_adjoint(const ora_cfg *c, cplx *psi) { cn_x_impl(c, psi, 1); }
void ora_cn_y_adjoint(const ora_cfg *c, cplx *psi) { cn_y_impl(c, psi, 1); }
