/*
 * Plain FP64 CPU oracle of the boosted-frame FDTD/PIC time step of MITHRA
 * (Fallahi, Yahaghi, Kaertner, arXiv:1612.03310, chapter "Methodology").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the GPU library.
 *
 * Everything is in SI units and double precision, with plain scalar loops in
 * the order the paper describes the method.  No blocking, fusion or
 * reordering beyond what the equations state.
 *
 * Readings of the paper taken here (each one is also listed in the design
 * notes of the repository):
 *   R1  the coefficient alpha'_6 = alpha'_7 of eq. (updateEquation) carries
 *       -2A(c dt/dx)^2 - 2A(c dt/dy)^2 (the printed second dx is dy);
 *   R2  source signs follow eqs. (HelmholtzA), (HelmholtzF):
 *       A^{n+1} += (c dt)^2 mu0 J,  phi^{n+1} += (c dt)^2 rho / eps0;
 *   R3  the n+1 term of B_z uses A_y on both sides;
 *   R4  interpolation weights are the standard linear (cloud-in-cell)
 *       weights 1-f and f;
 *   R5  rho and phi live on vertices, A_l and J_l on the l-edges
 *       (A_x at (i+1/2, j, k), ...; along l that grid has one point fewer,
 *       so all grids span the same box); the vertex value of A_l used in the
 *       E, B formulas is the mean of the two adjacent edge samples; the
 *       current is deposited with Esirkepov's density decomposition so
 *       that discrete charge continuity holds;
 *   R6  with N > 1 particle sub-steps, the grid field is interpolated once
 *       at the start position (where and when it is centred) and held;
 *       the undulator field is evaluated at every sub-step;
 *   R8  rest-frame undulator field: E_x = -g0 b0 c B'_y, B_y = g0 B'_y,
 *       B_z = B'_z, phase k_u z' with z' = g0 (z - z_e + b0 c t);
 *   R10 start from zero potentials, J^0 = 0, rho^{1/2} from the input
 *       positions (taken as r^{1/2}; momenta half a particle sub-step
 *       earlier, u^0 with one sub-step);
 *   R16 first-order Mur on faces, then edges, then corners; a point on
 *       several faces uses the rule of its highest-priority axis
 *       (z > y > x);
 *   R19 second-order Mur: on faces the printed update with gamma_0..12
 *       (those coefficients discretise the condition with +c/2 times the
 *       transverse Laplacian, the standard form; the printed equation's
 *       minus sign is read as a typo).  On edges and corners the face
 *       conditions involved, written in the inward coordinate s of each
 *       face, are added and discretised at the centre of the edge square or
 *       corner cube; the second derivatives along the face normals, which
 *       would need points outside the domain, are replaced through the wave
 *       equation, leaving
 *         edge:   (d_sa + d_sb) d_t xi - 3/(2c) d_tt xi + c/2 d_ee xi = 0,
 *         corner: (d_sa + d_sb + d_sc) d_t xi - 2/c d_tt xi = 0;
 *       faces first, then edges, then corners;
 *   R20 seed (section "Seed Field"): a plane wave of vector potential
 *       travelling towards +z, A = A0 p s(t - (z - z_ref)/c) with p in the
 *       x-y plane and s one of the printed signal shapes, is brought in by
 *       the TF/SF corrections at the second (scattered-field) and third
 *       (total-field) planes after the z_min boundary.  The corrections take
 *       the standard signs, so that the total-field region carries +A; the
 *       printed signs would inject -A.  The printed "sinusoidal pulse" is
 *       the job file's "flat-top" signal;
 *   R17 a particle whose cell leaves [2, n_d - 3] on any axis is lost;
 *   R21 bunching factor (section "Bunching factor"), a diagnostic here:
 *       b_h = |<exp(i h K z)>| over live particles, K = 2 gamma0 k_u;
 *   R22 power at the harmonics h omega_1 (omega_1 = gamma0 beta0 c k_u)
 *       through the power plane from a running DFT of the plane's fields
 *       (section "FEL-OUTPUT" names the output, not its transform);
 *   R24 optical undulator (section "UNDULATOR"): a plane wave towards -z,
 *       A_perp = a p s(t + (z - z_ref)/c) in the rest frame with the seed's
 *       signal shapes, in place of the static undulator's field on the
 *       particles;
 *   R25 its Gaussian-beam type: the same wave with the paraxial envelope of
 *       an astigmatic Gaussian beam focused at r_f, Rayleigh lengths z_par
 *       (along p) and z_perp (along z x p), carrier wave number k = 2 pi f/c:
 *       A_perp = a p Re{U S(t + (z - z_ref)/c)}, S the analytic signal of s
 *       (envelope times exp(i(w x + cep))), U = u(xi, z_par) u(eta, z_perp),
 *       u(v, zr) = sqrt(i zr / q) exp(-i k v^2 / (2 q)), q = zeta + i zr,
 *       zeta = z_f - z; fields E = -dA/dt, B = curl A (no scalar potential).
 *       The seed's Gaussian-beam type is the same beam towards +z
 *       (zeta = z - z_f, argument t - (z - z_ref)/c) injected point by point
 *       through the TF/SF planes.
 */
#include <assert.h>
#include <complex.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#undef I /* loops use I, J, K as vertex indices; the imaginary unit is ORC_J */
#define ORC_J _Complex_I
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 */
#define ORC_C 299792458.0
#define ORC_QE 1.602176634e-19
#define ORC_ME 9.1093837015e-31
#define ORC_EPS0 8.8541878128e-12
#define ORC_MU0 (1.0 / (ORC_EPS0 * ORC_C * ORC_C))
#define ORC_PI 3.14159265358979323846

#define ORC_NDIAG 29
#define ORC_MAXF 32 /* normalized frequencies of the plane spectrum */

typedef struct orc_sim {
    int n[3];
    double d[3], o[3];
    double nu, A;
    int N, sc, bc[3]; /* bc: 0 = Mur absorbing boundary, 1 = periodic */
    int mur2;         /* the Mur boundaries are of second order */
    /* seed plane wave (reading R20) */
    int seed_on, seed_sig;
    double seed_a0, seed_p[2], seed_f, seed_t0, seed_tau, seed_cep, seed_zref;
    /* its beam (reading R25): 0 plane wave, 1 Gaussian beam along +z */
    int seed_beam;
    double seed_zr[2], seed_focus[3];
    /* optical undulator (reading R24): a plane wave towards -z in place of the
       static undulator, same signal shapes as the seed */
    int opt_on, opt_sig;
    double opt_a, opt_p[2], opt_f, opt_t0, opt_tau, opt_cep, opt_zref;
    /* its beam (reading R25): 0 plane wave, 1 Gaussian beam with Rayleigh
       lengths along p and along z x p, focused at opt_focus */
    int opt_beam;
    double opt_zr[2], opt_focus[3];
    double lambda_u, K, gamma_beam, z_e;
    double und_len; /* lab length of the static undulator from z' = 0; <= 0: unbounded */
    /* derived constants */
    double dt, dtb, a1, a2, a4, a6, a8;
    double mur[3][5];
    double gamma0, beta0, B0, ku;
    /* mesh arrays, n[0]*n[1]*n[2] doubles each, x fastest */
    long ncell;
    double *pot[3][4]; /* [level slot][Ax, Ay, Az, phi] */
    int lprev, lcur, lnext;
    double *J[3], *rho, *rho_prev, *bg;
    double *E[3], *B[3];
    /* particles */
    long np;
    double *x, *u, *x_old;
    unsigned char *alive;
    double q, m;
    long step, lost;
    int nonfinite_u;
    /* diagnostics */
    int probe[3], kp;
    int kp_extra[3]; /* further sampling plates (-1: none), power only */
    double *diag;
    long ndiag, cap;
    /* running DFT of Ex, Ey, Bx, By on the power plane at nu_f omega_1
       (reading R22; f < nfreq, nu = 1, 2, 3 unless set): per plane point and
       frequency 4 complex sums, restarted when particles are loaded */
    int nfreq;
    double fnu[ORC_MAXF];
    double *spec;
    long nspec;
    /* per row: the mean power at each frequency since the restart, rest
       frame then lab frame (2 nfreq doubles) */
    double *srow;
} orc_sim;

/* ---- indexing ---------------------------------------------------------- */

static inline long wrap(const orc_sim *s, int a, int i)
{
    int n = s->n[a];
    if (i >= 0 && i < n) return i;
    if (!s->bc[a]) abort(); /* an out-of-range read is an oracle bug */
    return i < 0 ? i + n : i - n; /* periodic axis; offsets are at most 1 */
}

static inline long IX(const orc_sim *s, int i, int j, int k)
{
    long ii = wrap(s, 0, i);
    long jj = wrap(s, 1, j);
    long kk = wrap(s, 2, k);
    return (kk * s->n[1] + jj) * s->n[0] + ii;
}

/* range of vertices where the E, B formulas are evaluated: [1, n-2] on a
   Mur axis, every point on a periodic axis */
static void interior(const orc_sim *s, int d, int *lo, int *hi)
{
    if (s->bc[d]) { *lo = 0; *hi = s->n[d] - 1; }
    else { *lo = 1; *hi = s->n[d] - 2; }
}

/* number of points of component c's grid along axis a (reading R5): the
   l-edge grid of A_l and J_l has one point fewer than the vertex grid along
   l, so every grid spans the same box [0, (n-1) d]; the last layer of the
   array is then unused.  On a periodic axis all n points are used. */
static int extent(const orc_sim *s, int c, int a)
{
    return (c == a && !s->bc[a]) ? s->n[a] - 1 : s->n[a];
}

/* ---- set-up: constants of eqs. (updateEquation), (NSFDCoefficient),
        the first-order Mur coefficients, and the Lorentz boost ----------- */

orc_sim *orc_create(const int n[3], const double d[3], const double origin[3],
                    double courant, double nsfd_A, int substeps, int space_charge,
                    const int bc[3], double lambda_u, double K, double gamma_beam,
                    double z_e)
{
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    for (int a = 0; a < 3; a++) {
        s->n[a] = n[a];
        s->d[a] = d[a];
        s->o[a] = origin[a];
        s->bc[a] = bc[a] == 1;
    }
    /* input codes per axis: 0 first-order Mur, 1 periodic, 2 second-order Mur;
       the absorbing axes share one order */
    {
        int has1 = 0, has2 = 0;
        for (int a = 0; a < 3; a++) {
            has1 |= bc[a] == 0;
            has2 |= bc[a] == 2;
        }
        if (has1 && has2) abort();
        s->mur2 = has2;
    }
    s->nu = courant;
    s->N = substeps;
    s->sc = space_charge;
    s->lambda_u = lambda_u;
    s->K = K;
    s->gamma_beam = gamma_beam;
    s->z_e = z_e;

    double dx = d[0], dy = d[1], dz = d[2];
    /* time step from the longitudinal cell and the Courant number */
    s->dt = courant * dz / ORC_C;
    s->dtb = s->dt / substeps;
    /* eq. (NSFDCoefficient) unless an explicit A is given */
    if (nsfd_A < 0.0)
        s->A = 0.25 * (1.0 + 0.02 / ((dz / dx) * (dz / dx) + (dz / dy) * (dz / dy)));
    else
        s->A = nsfd_A;
    double nx2 = (ORC_C * s->dt / dx) * (ORC_C * s->dt / dx);
    double ny2 = (ORC_C * s->dt / dy) * (ORC_C * s->dt / dy);
    double nz2 = (ORC_C * s->dt / dz) * (ORC_C * s->dt / dz);
    /* coefficients alpha' of eq. (updateEquation), reading R1 */
    s->a1 = 2.0 * (1.0 - (1.0 - 2.0 * s->A) * nx2 - (1.0 - 2.0 * s->A) * ny2 - nz2);
    s->a2 = nx2;
    s->a4 = ny2;
    s->a6 = nz2 - 2.0 * s->A * nx2 - 2.0 * s->A * ny2;
    s->a8 = (ORC_C * s->dt) * (ORC_C * s->dt);
    /* first-order Mur coefficients beta_0..beta_4, per face axis */
    for (int a = 0; a < 3; a++) {
        double cdt = ORC_C * s->dt, h = d[a];
        s->mur[a][0] = (cdt - h) / (cdt + h);
        s->mur[a][1] = 2.0 * h / (cdt + h);
        s->mur[a][2] = -1.0;
        s->mur[a][3] = 2.0 * h / (cdt + h);
        s->mur[a][4] = (cdt - h) / (cdt + h);
    }
    /* average Lorentz factor in the undulator and the frame velocity */
    s->gamma0 = gamma_beam / sqrt(1.0 + K * K / 2.0);
    s->beta0 = sqrt(1.0 - 1.0 / (s->gamma0 * s->gamma0));
    /* K = e B0 lambda_u / (2 pi m c) */
    s->B0 = 2.0 * ORC_PI * ORC_ME * ORC_C * K / (ORC_QE * lambda_u);
    s->ku = 2.0 * ORC_PI / lambda_u;

    s->ncell = (long)n[0] * n[1] * n[2];
    for (int l = 0; l < 3; l++)
        for (int c = 0; c < 4; c++)
            s->pot[l][c] = (double *)calloc(s->ncell, sizeof(double));
    s->lprev = 0;
    s->lcur = 1;
    s->lnext = 2;
    for (int c = 0; c < 3; c++) {
        s->J[c] = (double *)calloc(s->ncell, sizeof(double));
        s->E[c] = (double *)calloc(s->ncell, sizeof(double));
        s->B[c] = (double *)calloc(s->ncell, sizeof(double));
    }
    s->rho = (double *)calloc(s->ncell, sizeof(double));
    s->rho_prev = (double *)calloc(s->ncell, sizeof(double));
    s->bg = NULL;
    s->probe[0] = n[0] / 2;
    s->probe[1] = n[1] / 2;
    s->probe[2] = n[2] / 2;
    s->kp = n[2] / 2;
    for (int e = 0; e < 3; e++) s->kp_extra[e] = -1;
    s->cap = 1024;
    s->diag = (double *)malloc(sizeof(double) * ORC_NDIAG * s->cap);
    s->nfreq = 3;
    for (int f = 0; f < 3; f++) s->fnu[f] = f + 1.0;
    s->spec = (double *)calloc((size_t)n[0] * n[1] * 8 * s->nfreq, sizeof(double));
    s->nspec = 0;
    s->srow = (double *)malloc(sizeof(double) * 2 * ORC_MAXF * s->cap);
    s->und_len = 0.0;
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    for (int l = 0; l < 3; l++)
        for (int c = 0; c < 4; c++) free(s->pot[l][c]);
    for (int c = 0; c < 3; c++) {
        free(s->J[c]);
        free(s->E[c]);
        free(s->B[c]);
    }
    free(s->rho);
    free(s->rho_prev);
    free(s->bg);
    free(s->x);
    free(s->u);
    free(s->x_old);
    free(s->alive);
    free(s->diag);
    free(s->spec);
    free(s->srow);
    free(s);
}

/* static neutralising background charge (test fixture, not in the paper) */
void orc_set_background(orc_sim *s, const double *bg)
{
    if (!s->bg) s->bg = (double *)calloc(s->ncell, sizeof(double));
    memcpy(s->bg, bg, sizeof(double) * s->ncell);
}

void orc_config_diag(orc_sim *s, int pi, int pj, int pk, int kp)
{
    s->probe[0] = pi;
    s->probe[1] = pj;
    s->probe[2] = pk;
    s->kp = kp;
}

/* Normalized frequencies of the plane spectrum (section "FEL-OUTPUT":
   normalized-frequency, or a sweep from the minimum to the maximum at the
   given resolution), nu_f = omega_f / omega_1; the running DFT restarts. */
void orc_set_spectrum(orc_sim *s, const double *nu, int nfreq)
{
    if (nfreq < 1 || nfreq > ORC_MAXF) abort();
    s->nfreq = nfreq;
    for (int f = 0; f < nfreq; f++) s->fnu[f] = nu[f];
    free(s->spec);
    s->spec = (double *)calloc((size_t)s->n[0] * s->n[1] * 8 * nfreq, sizeof(double));
    s->nspec = 0;
}

/* Total lab length of the static undulator (section "UNDULATOR", length),
   a whole number of periods; <= 0 leaves it unbounded. */
void orc_set_undulator_length(orc_sim *s, double length) { s->und_len = length; }

/* Further sampling plates (section "FEL-OUTPUT": the plate distance may be
   repeated): the radiated power through planes k1..k3, -1 for none. */
void orc_config_extra_planes(orc_sim *s, int k1, int k2, int k3)
{
    s->kp_extra[0] = k1;
    s->kp_extra[1] = k2;
    s->kp_extra[2] = k3;
}

/* ---- cloud-in-cell weights (eq. (fieldInterpolation), reading R4) ------ */

static void cell_of(const orc_sim *s, const double *x, int c[3], double f[3])
{
    for (int a = 0; a < 3; a++) {
        double xi = (x[a] - s->o[a]) / s->d[a];
        double fl = floor(xi);
        c[a] = (int)fl;
        f[a] = xi - fl;
    }
}

static int inside(const orc_sim *s, const int c[3])
{
    for (int a = 0; a < 3; a++)
        if (c[a] < 2 || c[a] > s->n[a] - 3) return 0;
    return 1;
}

/* ---- charge and current deposition ------------------------------------- */

/* charge density of one macro-particle spread to the 8 vertices of its cell,
   rho = q / (dx dy dz) times the linear weights (section "Current
   Deposition") */
static void deposit_rho(orc_sim *s, double *rho, const double *x)
{
    int c[3];
    double f[3];
    cell_of(s, x, c, f);
    double q_dv = s->q / (s->d[0] * s->d[1] * s->d[2]);
    for (int K = 0; K < 2; K++)
        for (int J = 0; J < 2; J++)
            for (int I = 0; I < 2; I++) {
                double w = (I ? f[0] : 1.0 - f[0]) * (J ? f[1] : 1.0 - f[1]) *
                           (K ? f[2] : 1.0 - f[2]);
                rho[IX(s, c[0] + I, c[1] + J, c[2] + K)] += q_dv * w;
            }
}

/* current of one macro-particle moving from x0 (time n+1/2) to x1 (time
   n+3/2), eq. (currentIntegral) with reading R5: Esirkepov's decomposition
   of the change of the linear-weight density into three directional parts
   W^x, W^y, W^z; J_l on the l-edges is minus the running sum of W^l along l,
   scaled by q dl / (dV dt). */
void orc_deposit_current(orc_sim *s, const double *x0, const double *x1)
{
    int c0[3], c1[3], base[3];
    double f0[3], f1[3];
    cell_of(s, x0, c0, f0);
    cell_of(s, x1, c1, f1);
    double S0[3][3], DS[3][3];
    for (int a = 0; a < 3; a++) {
        /* the 3-point shape arrays below hold a move of at most one cell per
           axis: a particle moves less than c dt per field step, and
           c dt <= d_a on every mesh the library accepts (nu <= 1 with the
           stability condition dz < dx, dy) */
        assert(c1[a] - c0[a] >= -1 && c1[a] - c0[a] <= 1);
        base[a] = c0[a] < c1[a] ? c0[a] : c1[a];
        double s1[3] = {0.0, 0.0, 0.0};
        for (int m = 0; m < 3; m++) S0[a][m] = 0.0;
        S0[a][c0[a] - base[a]] += 1.0 - f0[a];
        S0[a][c0[a] - base[a] + 1] += f0[a];
        s1[c1[a] - base[a]] += 1.0 - f1[a];
        s1[c1[a] - base[a] + 1] += f1[a];
        for (int m = 0; m < 3; m++) DS[a][m] = s1[m] - S0[a][m];
    }
    double dV = s->d[0] * s->d[1] * s->d[2];
    /* W^l at the 3x3x3 vertices of the box starting at base */
    for (int l = 0; l < 3; l++) {
        int p = (l + 1) % 3, r = (l + 2) % 3; /* the two other axes */
        double unit = s->q * s->d[l] / (dV * s->dt);
        for (int b = 0; b < 3; b++)
            for (int e = 0; e < 3; e++) {
                double run = 0.0;
                for (int a = 0; a < 2; a++) { /* edge (base+a) + 1/2 */
                    double W = DS[l][a] * (S0[p][b] * S0[r][e] + 0.5 * DS[p][b] * S0[r][e] +
                                           0.5 * S0[p][b] * DS[r][e] +
                                           DS[p][b] * DS[r][e] / 3.0);
                    run += W;
                    int v[3];
                    v[l] = base[l] + a;
                    v[p] = base[p] + b;
                    v[r] = base[r] + e;
                    s->J[l][IX(s, v[0], v[1], v[2])] += -unit * run;
                }
            }
    }
}

/* ---- particles ----------------------------------------------------------- */

int orc_set_particles(orc_sim *s, long np, const double *x, const double *u, double q,
                      double m)
{
    free(s->x);
    free(s->u);
    free(s->x_old);
    free(s->alive);
    s->np = np;
    s->q = q;
    s->m = m;
    s->x = (double *)malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    s->u = (double *)malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    s->x_old = (double *)malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    s->alive = (unsigned char *)malloc(np > 0 ? np : 1);
    memcpy(s->x, x, sizeof(double) * 3 * np);
    memcpy(s->u, u, sizeof(double) * 3 * np);
    memcpy(s->x_old, x, sizeof(double) * 3 * np);
    s->lost = 0;
    /* reading R10: rho^{1/2} from the initial positions, J^0 = 0 */
    memset(s->rho, 0, sizeof(double) * s->ncell);
    for (int c = 0; c < 3; c++) memset(s->J[c], 0, sizeof(double) * s->ncell);
    for (long p = 0; p < np; p++) {
        int c[3];
        double f[3];
        cell_of(s, &s->x[3 * p], c, f);
        s->alive[p] = (unsigned char)inside(s, c);
        if (!s->alive[p]) { s->lost++; continue; }
        deposit_rho(s, s->rho, &s->x[3 * p]);
    }
    memcpy(s->rho_prev, s->rho, sizeof(double) * s->ncell);
    /* the plane spectrum is a mean since the particles were loaded */
    memset(s->spec, 0, sizeof(double) * (size_t)s->n[0] * s->n[1] * 8 * s->nfreq);
    s->nspec = 0;
    return 0;
}

/* ---- O2: potential update, eq. (updateEquation) -------------------------- */

static void boundary_mur1(orc_sim *s, int comp);
static void boundary_mur2(orc_sim *s, int comp);
static void seed_tfsf(orc_sim *s, int c, const int lo[3], const int hi[3]);

void orc_field_update(orc_sim *s)
{
    double A = s->A;
    for (int c = 0; c < 4; c++) {
        double *P = s->pot[s->lcur][c], *Q = s->pot[s->lprev][c], *R = s->pot[s->lnext][c];
        if (c == 3 && !s->sc) {
            memset(R, 0, sizeof(double) * s->ncell);
            continue;
        }
        /* interior points of this component's grid: [1, extent-2] on a Mur
           axis, all points on a periodic axis */
        int lo[3], hi[3];
        for (int a = 0; a < 3; a++) {
            lo[a] = s->bc[a] ? 0 : 1;
            hi[a] = s->bc[a] ? s->n[a] - 1 : extent(s, c, a) - 2;
        }
#pragma omp parallel for schedule(static)
        for (int k = lo[2]; k <= hi[2]; k++)
            for (int j = lo[1]; j <= hi[1]; j++)
                for (int i = lo[0]; i <= hi[0]; i++) {
                    long p = IX(s, i, j, k);
                    /* z-weighted transverse neighbours, eq. (NSFDtrick) */
                    double bxp = A * P[IX(s, i + 1, j, k - 1)] + (1.0 - 2.0 * A) * P[IX(s, i + 1, j, k)] +
                                 A * P[IX(s, i + 1, j, k + 1)];
                    double bxm = A * P[IX(s, i - 1, j, k - 1)] + (1.0 - 2.0 * A) * P[IX(s, i - 1, j, k)] +
                                 A * P[IX(s, i - 1, j, k + 1)];
                    double byp = A * P[IX(s, i, j + 1, k - 1)] + (1.0 - 2.0 * A) * P[IX(s, i, j + 1, k)] +
                                 A * P[IX(s, i, j + 1, k + 1)];
                    double bym = A * P[IX(s, i, j - 1, k - 1)] + (1.0 - 2.0 * A) * P[IX(s, i, j - 1, k)] +
                                 A * P[IX(s, i, j - 1, k + 1)];
                    /* source term, signs of reading R2 */
                    double zeta;
                    if (c < 3)
                        zeta = ORC_MU0 * s->J[c][p];
                    else
                        zeta = (s->rho[p] + (s->bg ? s->bg[p] : 0.0)) / ORC_EPS0;
                    R[p] = -Q[p] + s->a1 * P[p] + s->a2 * bxp + s->a2 * bxm + s->a4 * byp +
                           s->a4 * bym + s->a6 * P[IX(s, i, j, k + 1)] + s->a6 * P[IX(s, i, j, k - 1)] +
                           s->a8 * zeta;
                }
        seed_tfsf(s, c, lo, hi);
        if (s->mur2) boundary_mur2(s, c);
        else boundary_mur1(s, c);
    }
}

/* ---- O2b: seed plane wave by the TF/SF technique (section "Seed Field",
        reading R20) ------------------------------------------------------- */

/* the printed signal shapes; x = t - t0 */
double orc_seed_signal(const orc_sim *s, double t)
{
    double x = t - s->seed_t0, ln2 = log(2.0), tau = s->seed_tau;
    double carrier = cos(2.0 * ORC_PI * s->seed_f * x + s->seed_cep);
    double g = exp(-2.0 * ln2 * x * x / (tau * tau));
    switch (s->seed_sig) {
    case 0: /* modulated Neumann */
        return -s->seed_a0 * 4.0 * ln2 * carrier * x / (tau * tau) * g;
    case 1: /* modulated Gaussian */
        return s->seed_a0 * carrier * g;
    case 2: /* modulated hyperbolic secant */
        return s->seed_a0 * carrier / cosh(x / tau);
    default: /* sinusoidal pulse: Gaussian rise, then the bare carrier */
        return s->seed_a0 * carrier * (x <= 0.0 ? g : 1.0);
    }
}

void orc_set_seed(orc_sim *s, int on, double a0, double px, double py, double freq, double t0,
                  double tau, double cep, int signal, double z_ref)
{
    s->seed_on = on;
    s->seed_a0 = a0;
    s->seed_p[0] = px;
    s->seed_p[1] = py;
    s->seed_f = freq;
    s->seed_t0 = t0;
    s->seed_tau = tau;
    s->seed_cep = cep;
    s->seed_sig = signal;
    s->seed_zref = z_ref;
}

static double complex analytic_signal(int sig, double a, double f, double t0, double tau,
                                      double cep, double t, double complex *rate);

void orc_set_seed_beam(orc_sim *s, int beam, double zr_par, double zr_perp, double xf, double yf,
                       double zf)
{
    s->seed_beam = beam;
    s->seed_zr[0] = zr_par;
    s->seed_zr[1] = zr_perp;
    s->seed_focus[0] = xf;
    s->seed_focus[1] = yf;
    s->seed_focus[2] = zf;
}

/* incident potential component c at the grid point (i, j, k) of that
   component (A_x sits at x + dx/2, A_y at y + dy/2), time level n: the plane
   wave, or for the Gaussian-beam seed (reading R25, travelling towards +z,
   zeta = z - z_f) Re{U S} with the analytic signal S */
static double seed_incident(const orc_sim *s, int c, int i, int j, int k, double t)
{
    double z = s->o[2] + k * s->d[2];
    double tt = t - (z - s->seed_zref) / ORC_C;
    if (s->seed_beam != 1) return s->seed_p[c] * orc_seed_signal(s, tt);
    double x = s->o[0] + (i + (c == 0 ? 0.5 : 0.0)) * s->d[0];
    double y = s->o[1] + (j + (c == 1 ? 0.5 : 0.0)) * s->d[1];
    double k0 = 2.0 * ORC_PI * s->seed_f / ORC_C, px = s->seed_p[0], py = s->seed_p[1];
    double pn = sqrt(px * px + py * py);
    double X = x - s->seed_focus[0], Y = y - s->seed_focus[1], zeta = z - s->seed_focus[2];
    double xi = (X * px + Y * py) / pn, eta = (-X * py + Y * px) / pn;
    double complex q1 = zeta + ORC_J * s->seed_zr[0], q2 = zeta + ORC_J * s->seed_zr[1];
    double complex U = csqrt(ORC_J * s->seed_zr[0] / q1) * csqrt(ORC_J * s->seed_zr[1] / q2) *
                       cexp(-ORC_J * k0 * xi * xi / (2.0 * q1) - ORC_J * k0 * eta * eta / (2.0 * q2));
    double complex rate;
    double complex S = analytic_signal(s->seed_sig, s->seed_a0, s->seed_f, s->seed_t0, s->seed_tau,
                                       s->seed_cep, tt, &rate);
    return s->seed_p[c] * creal(U * S);
}

double orc_seed_incident(const orc_sim *s, int c, int i, int j, int k, double t)
{
    return seed_incident(s, c, i, j, k, t);
}

/* after the interior update of component c (A_x or A_y): the scattered-field
   plane k_s = 2 loses what its update took from the incident field on the
   total-field plane k_t = 3, and k_t gains what its update missed on k_s */
static void seed_tfsf(orc_sim *s, int c, const int lo[3], const int hi[3])
{
    if (!s->seed_on || c > 1 || s->seed_p[c] == 0.0) return;
    double *R = s->pot[s->lnext][c];
    double t = s->step * s->dt, A = s->A;
    const int ks = 2, kt = 3;
    for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
            /* the neighbours on the other plane, as in eq. (updateEquation)
               (all equal for the plane wave) */
            double ft_ip = seed_incident(s, c, i + 1, j, kt, t), ft_im = seed_incident(s, c, i - 1, j, kt, t);
            double ft_jp = seed_incident(s, c, i, j + 1, kt, t), ft_jm = seed_incident(s, c, i, j - 1, kt, t);
            double fs_ip = seed_incident(s, c, i + 1, j, ks, t), fs_im = seed_incident(s, c, i - 1, j, ks, t);
            double fs_jp = seed_incident(s, c, i, j + 1, ks, t), fs_jm = seed_incident(s, c, i, j - 1, ks, t);
            R[IX(s, i, j, ks)] -= A * (s->a2 * ft_ip + s->a2 * ft_im + s->a4 * ft_jp + s->a4 * ft_jm) +
                                  s->a6 * seed_incident(s, c, i, j, kt, t);
            R[IX(s, i, j, kt)] += A * (s->a2 * fs_ip + s->a2 * fs_im + s->a4 * fs_jp + s->a4 * fs_jm) +
                                  s->a6 * seed_incident(s, c, i, j, ks, t);
        }
}

/* ---- O3: first-order Mur boundary, staged as reading R16 ----------------- */

static void boundary_mur1(orc_sim *s, int c)
{
    double *P = s->pot[s->lcur][c], *Q = s->pot[s->lprev][c], *R = s->pot[s->lnext][c];
    int ext[3];
    for (int a = 0; a < 3; a++) ext[a] = extent(s, c, a);
    /* a point of one stage reads only points of earlier stages */
    for (int stage = 1; stage <= 3; stage++)
#pragma omp parallel for schedule(static)
        for (int k = 0; k < ext[2]; k++)
            for (int j = 0; j < ext[1]; j++)
                for (int i = 0; i < ext[0]; i++) {
                    int v[3] = {i, j, k}, nb = 0, top = -1;
                    for (int a = 0; a < 3; a++)
                        if (!s->bc[a] && (v[a] == 0 || v[a] == ext[a] - 1)) {
                            nb++;
                            top = a; /* highest axis wins: z > y > x */
                        }
                    if (nb != stage) continue;
                    int w[3] = {i, j, k};
                    w[top] += (v[top] == 0) ? 1 : -1; /* inward neighbour */
                    long p = IX(s, v[0], v[1], v[2]), q = IX(s, w[0], w[1], w[2]);
                    const double *b = s->mur[top];
                    R[p] = b[0] * Q[p] + b[1] * P[p] + b[2] * Q[q] + b[3] * P[q] + b[4] * R[q];
                }
}

/* ---- O3b: second-order Mur boundary (section "Boundary Truncation"),
        faces with the printed gamma coefficients, edges and corners by
        reading R19 --------------------------------------------------------- */

/* face normal to axis a (either side): transverse axes u < v */
static void mur2_face(orc_sim *s, int c, const int v[3], int a)
{
    const double *P = s->pot[s->lcur][c], *Q = s->pot[s->lprev][c];
    double *R = s->pot[s->lnext][c];
    int u = (a == 0) ? 1 : 0, w = (a == 2) ? 1 : 2;
    double cdt = ORC_C * s->dt, h = s->d[a];
    double ru = cdt / s->d[u], rw = cdt / s->d[w];
    double g0 = (cdt - h) / (cdt + h), g4 = g0;
    double g1 = h * (2.0 - rw * rw - ru * ru) / (cdt + h), g3 = g1;
    double g2 = -1.0;
    double gu = ru * ru * h / (2.0 * (cdt + h)); /* gamma_5, 6, 9, 10 */
    double gw = rw * rw * h / (2.0 * (cdt + h)); /* gamma_7, 8, 11, 12 */
    int in[3] = {v[0], v[1], v[2]};
    in[a] += (v[a] == 0) ? 1 : -1; /* the layer inside */
    int bp[3], bm[3], ip[3], im[3];
    double tb = 0.0, ti = 0.0; /* transverse neighbours at level n, boundary / inner layer */
    for (int t = 0; t < 2; t++) {
        int ax = t ? w : u;
        double g = t ? gw : gu;
        memcpy(bp, v, sizeof bp);
        memcpy(bm, v, sizeof bm);
        memcpy(ip, in, sizeof ip);
        memcpy(im, in, sizeof im);
        bp[ax]++;
        bm[ax]--;
        ip[ax]++;
        im[ax]--;
        tb += g * (P[IX(s, bp[0], bp[1], bp[2])] + P[IX(s, bm[0], bm[1], bm[2])]);
        ti += g * (P[IX(s, ip[0], ip[1], ip[2])] + P[IX(s, im[0], im[1], im[2])]);
    }
    long p = IX(s, v[0], v[1], v[2]), q = IX(s, in[0], in[1], in[2]);
    R[p] = g0 * Q[p] + g1 * P[p] + g2 * Q[q] + g3 * P[q] + g4 * R[q] + ti + tb;
}

/* the summed edge / corner condition of reading R19, discretised at the
   centre of the square (na = 2 face axes) or cube (na = 3) whose corner v is
   the unknown point, evaluated with the value x in place of xi^{n+1}(v) */
static double mur2_joint_residual(orc_sim *s, int c, const int v[3], const int ax[3], int na,
                                  double x)
{
    const double *P = s->pot[s->lcur][c], *Q = s->pot[s->lprev][c], *R = s->pot[s->lnext][c];
    double dt = s->dt;
    int npt = 1 << na;
    double sum_dt[3] = {0.0, 0.0, 0.0}, dtt = 0.0, dee = 0.0;
    int e = 3 - ax[0] - ax[1]; /* the edge direction (edges only) */
    for (int m = 0; m < npt; m++) {
        int pt[3] = {v[0], v[1], v[2]};
        for (int t = 0; t < na; t++) {
            int off = (m >> t) & 1;
            pt[ax[t]] += off * ((v[ax[t]] == 0) ? 1 : -1);
        }
        long p = IX(s, pt[0], pt[1], pt[2]);
        double rn = (m == 0) ? x : R[p];
        /* d_s d_t: inner minus outer layer along each face normal */
        for (int t = 0; t < na; t++) {
            double sgn = ((m >> t) & 1) ? 1.0 : -1.0;
            sum_dt[t] += sgn * (rn - Q[p]);
        }
        dtt += rn - 2.0 * P[p] + Q[p];
        if (na == 2) {
            int pe[3], me[3];
            memcpy(pe, pt, sizeof pe);
            memcpy(me, pt, sizeof me);
            pe[e]++;
            me[e]--;
            dee += P[IX(s, pe[0], pe[1], pe[2])] - 2.0 * P[p] + P[IX(s, me[0], me[1], me[2])];
        }
    }
    /* averages over the points of the square / cube */
    double inv = 1.0 / npt, pairs = 2.0 / npt;
    double res = 0.0;
    for (int t = 0; t < na; t++) res += sum_dt[t] * pairs / (2.0 * dt * s->d[ax[t]]);
    dtt *= inv / (dt * dt);
    if (na == 2) {
        dee *= inv / (s->d[e] * s->d[e]);
        res += -3.0 / (2.0 * ORC_C) * dtt + 0.5 * ORC_C * dee;
    } else {
        res += -2.0 / ORC_C * dtt;
    }
    return res;
}

static void boundary_mur2(orc_sim *s, int c)
{
    double *R = s->pot[s->lnext][c];
    int ext[3];
    for (int a = 0; a < 3; a++) ext[a] = extent(s, c, a);
    /* a point of one stage reads only points of earlier stages */
    for (int stage = 1; stage <= 3; stage++)
#pragma omp parallel for schedule(static)
        for (int k = 0; k < ext[2]; k++)
            for (int j = 0; j < ext[1]; j++)
                for (int i = 0; i < ext[0]; i++) {
                    int v[3] = {i, j, k}, ax[3], nb = 0;
                    for (int a = 0; a < 3; a++)
                        if (!s->bc[a] && (v[a] == 0 || v[a] == ext[a] - 1)) ax[nb++] = a;
                    if (nb != stage) continue;
                    if (nb == 1) {
                        mur2_face(s, c, v, ax[0]);
                    } else {
                        /* linear in the unknown: solve r(0) + (r(1) - r(0)) x = 0 */
                        double r0 = mur2_joint_residual(s, c, v, ax, nb, 0.0);
                        double r1 = mur2_joint_residual(s, c, v, ax, nb, 1.0);
                        R[IX(s, v[0], v[1], v[2])] = -r0 / (r1 - r0);
                    }
                }
}

/* ---- O4: E and B at the vertices at t_{n+1/2} ------------------------------ */

/* vertex value of the edge-sampled A_l: mean of the two adjacent edges */
static inline double abar(const orc_sim *s, const double *Al, int l, int i, int j, int k)
{
    int v[3] = {i, j, k};
    v[l] -= 1;
    return 0.5 * (Al[IX(s, i, j, k)] + Al[IX(s, v[0], v[1], v[2])]);
}

void orc_vertex_fields(orc_sim *s)
{
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) interior(s, a, &lo[a], &hi[a]);
    for (int c = 0; c < 3; c++) {
        memset(s->E[c], 0, sizeof(double) * s->ncell);
        memset(s->B[c], 0, sizeof(double) * s->ncell);
    }
    double *const *An = s->pot[s->lcur];
    double *const *An1 = s->pot[s->lnext];
    const double *phi = s->pot[s->lcur][3];
    double dx = s->d[0], dy = s->d[1], dz = s->d[2], dt = s->dt;
#pragma omp parallel for schedule(static)
    for (int k = lo[2]; k <= hi[2]; k++)
        for (int j = lo[1]; j <= hi[1]; j++)
            for (int i = lo[0]; i <= hi[0]; i++) {
                long p = IX(s, i, j, k);
                /* eq. (EvsA) discretised at the vertex */
                s->E[0][p] = -(abar(s, An1[0], 0, i, j, k) - abar(s, An[0], 0, i, j, k)) / dt -
                             (phi[IX(s, i + 1, j, k)] - phi[IX(s, i - 1, j, k)]) / (2.0 * dx);
                s->E[1][p] = -(abar(s, An1[1], 1, i, j, k) - abar(s, An[1], 1, i, j, k)) / dt -
                             (phi[IX(s, i, j + 1, k)] - phi[IX(s, i, j - 1, k)]) / (2.0 * dy);
                s->E[2][p] = -(abar(s, An1[2], 2, i, j, k) - abar(s, An[2], 2, i, j, k)) / dt -
                             (phi[IX(s, i, j, k + 1)] - phi[IX(s, i, j, k - 1)]) / (2.0 * dz);
                /* eq. (BvsA): mean of the central curls at levels n and n+1 */
                double bx = 0.0, by = 0.0, bz = 0.0;
                for (int lev = 0; lev < 2; lev++) {
                    double *const *Ap = lev ? An1 : An;
                    bx += (abar(s, Ap[2], 2, i, j + 1, k) - abar(s, Ap[2], 2, i, j - 1, k)) / (2.0 * dy) -
                          (abar(s, Ap[1], 1, i, j, k + 1) - abar(s, Ap[1], 1, i, j, k - 1)) / (2.0 * dz);
                    by += (abar(s, Ap[0], 0, i, j, k + 1) - abar(s, Ap[0], 0, i, j, k - 1)) / (2.0 * dz) -
                          (abar(s, Ap[2], 2, i + 1, j, k) - abar(s, Ap[2], 2, i - 1, j, k)) / (2.0 * dx);
                    bz += (abar(s, Ap[1], 1, i + 1, j, k) - abar(s, Ap[1], 1, i - 1, j, k)) / (2.0 * dx) -
                          (abar(s, Ap[0], 0, i, j + 1, k) - abar(s, Ap[0], 0, i, j - 1, k)) / (2.0 * dy);
                }
                s->B[0][p] = 0.5 * bx;
                s->B[1][p] = 0.5 * by;
                s->B[2][p] = 0.5 * bz;
            }
}

/* ---- O5: field at a particle, linear interpolation from the 8 vertices ---- */

void orc_gather(const orc_sim *s, const double *x, double *E, double *B)
{
    int c[3];
    double f[3];
    cell_of(s, x, c, f);
    for (int a = 0; a < 3; a++) E[a] = B[a] = 0.0;
    for (int K = 0; K < 2; K++)
        for (int J = 0; J < 2; J++)
            for (int I = 0; I < 2; I++) {
                double w = (I ? f[0] : 1.0 - f[0]) * (J ? f[1] : 1.0 - f[1]) *
                           (K ? f[2] : 1.0 - f[2]);
                long p = IX(s, c[0] + I, c[1] + J, c[2] + K);
                for (int a = 0; a < 3; a++) {
                    E[a] += w * s->E[a][p];
                    B[a] += w * s->B[a][p];
                }
            }
}

/* ---- O6: static planar undulator seen in the rest frame ------------------ */

/* Time derivative of the signal shapes of section "Seed Field" (the same
   four shapes as orc_seed_signal, amplitude a), differentiated by hand:
   carrier C = cos(w x + cep), envelope g = exp(-2 ln2 x^2 / tau^2). */
static double signal_rate(int sig, double a, double f, double t0, double tau, double cep, double t)
{
    double x = t - t0, ln2 = log(2.0), w = 2.0 * ORC_PI * f;
    double C = cos(w * x + cep), S = sin(w * x + cep);
    double g = exp(-2.0 * ln2 * x * x / (tau * tau));
    double g1 = -4.0 * ln2 * x / (tau * tau) * g;           /* g' */
    double g2 = -4.0 * ln2 / (tau * tau) * (g + x * g1);    /* g'' */
    switch (sig) {
    case 0: /* s = a C g' */
        return a * (-w * S * g1 + C * g2);
    case 1: /* s = a C g */
        return a * (-w * S * g + C * g1);
    case 2: { /* s = a C sech(x / tau) */
        double sech = 1.0 / cosh(x / tau);
        return a * (-w * S * sech - C * sech * tanh(x / tau) / tau);
    }
    default: /* Gaussian rise, then the bare carrier */
        return x <= 0.0 ? a * (-w * S * g + C * g1) : -a * w * S;
    }
}

/* The shapes as analytic signals: S = a e(x) exp(i(w x + cep)) with the
   envelope e of each shape, and dS/dt = a (e' + i w e) exp(i(w x + cep)).
   Their real parts are the signal and signal_rate. */
static double complex analytic_signal(int sig, double a, double f, double t0, double tau,
                                      double cep, double t, double complex *rate)
{
    double x = t - t0, ln2 = log(2.0), w = 2.0 * ORC_PI * f;
    double g = exp(-2.0 * ln2 * x * x / (tau * tau));
    double g1 = -4.0 * ln2 * x / (tau * tau) * g;
    double g2 = -4.0 * ln2 / (tau * tau) * (g + x * g1);
    double e, e1;
    switch (sig) {
    case 0: e = g1; e1 = g2; break;
    case 1: e = g; e1 = g1; break;
    case 2: e = 1.0 / cosh(x / tau); e1 = -e * tanh(x / tau) / tau; break;
    default: e = x <= 0.0 ? g : 1.0; e1 = x <= 0.0 ? g1 : 0.0; break;
    }
    double complex carrier = cexp(ORC_J * (w * x + cep));
    *rate = a * (e1 + ORC_J * w * e) * carrier;
    return a * e * carrier;
}

/* Gaussian-beam optical undulator (reading R25): E = -p dpsi/dt,
   B = grad psi x p = (-p_y dpsi/dz, p_x dpsi/dz, -|p| dpsi/deta) with
   psi = Re{U S}, xi and eta the distances along p/|p| and z x p/|p|;
   d/dz = (1/c) d/dt - d/dzeta. */
static void gaussian_beam_field(const orc_sim *s, double x, double y, double z, double t,
                                double *E, double *B)
{
    double k = 2.0 * ORC_PI * s->opt_f / ORC_C;
    double px = s->opt_p[0], py = s->opt_p[1];
    double pn = sqrt(px * px + py * py);
    double X = x - s->opt_focus[0], Y = y - s->opt_focus[1], zeta = s->opt_focus[2] - z;
    double xi = (X * px + Y * py) / pn, eta = (-X * py + Y * px) / pn;
    double complex q1 = zeta + ORC_J * s->opt_zr[0], q2 = zeta + ORC_J * s->opt_zr[1];
    double complex U = csqrt(ORC_J * s->opt_zr[0] / q1) * csqrt(ORC_J * s->opt_zr[1] / q2) *
                       cexp(-ORC_J * k * xi * xi / (2.0 * q1) - ORC_J * k * eta * eta / (2.0 * q2));
    double complex dU_deta = U * (-ORC_J * k * eta / q2);
    double complex dU_dzeta = U * (-1.0 / (2.0 * q1) + ORC_J * k * xi * xi / (2.0 * q1 * q1) -
                                   1.0 / (2.0 * q2) + ORC_J * k * eta * eta / (2.0 * q2 * q2));
    double complex rate;
    double complex S = analytic_signal(s->opt_sig, s->opt_a, s->opt_f, s->opt_t0, s->opt_tau,
                                       s->opt_cep, t + (z - s->opt_zref) / ORC_C, &rate);
    double dpsi_dt = creal(U * rate);
    double dpsi_dz = dpsi_dt / ORC_C - creal(dU_dzeta * S);
    double dpsi_deta = creal(dU_deta * S);
    E[0] = -px * dpsi_dt;
    E[1] = -py * dpsi_dt;
    E[2] = 0.0;
    B[0] = -py * dpsi_dz;
    B[1] = px * dpsi_dz;
    B[2] = -pn * dpsi_deta;
}

void orc_set_optical_beam(orc_sim *s, int beam, double zr_par, double zr_perp, double xf,
                          double yf, double zf)
{
    s->opt_beam = beam;
    s->opt_zr[0] = zr_par;
    s->opt_zr[1] = zr_perp;
    s->opt_focus[0] = xf;
    s->opt_focus[1] = yf;
    s->opt_focus[2] = zf;
}

void orc_set_optical(orc_sim *s, int on, double a, double px, double py, double freq, double t0,
                     double tau, double cep, int signal, double z_ref)
{
    s->opt_on = on;
    s->opt_a = a;
    s->opt_p[0] = px;
    s->opt_p[1] = py;
    s->opt_f = freq;
    s->opt_t0 = t0;
    s->opt_tau = tau;
    s->opt_cep = cep;
    s->opt_sig = signal;
    s->opt_zref = z_ref;
}

/* eqs. (undulatorField), fringe field for z' < 0, and the boost of reading R8;
   with the optical undulator on, the rest-frame plane wave
   A_perp = a p s(t + (z - z_ref)/c): E = -a p s', B = (-a p_y s'/c, a p_x s'/c, 0) */
void orc_undulator(const orc_sim *s, double x, double y, double z, double t, double *E,
                   double *B)
{
    if (s->opt_on && s->opt_beam == 1) {
        gaussian_beam_field(s, x, y, z, t, E, B);
        return;
    }
    if (s->opt_on) {
        double ds = signal_rate(s->opt_sig, s->opt_a, s->opt_f, s->opt_t0, s->opt_tau, s->opt_cep,
                                t + (z - s->opt_zref) / ORC_C);
        E[0] = -s->opt_p[0] * ds;
        E[1] = -s->opt_p[1] * ds;
        E[2] = 0.0;
        B[0] = -s->opt_p[1] * ds / ORC_C;
        B[1] = s->opt_p[0] * ds / ORC_C;
        B[2] = 0.0;
        return;
    }
    double zp = s->gamma0 * (z - s->z_e + s->beta0 * ORC_C * t); /* lab z' */
    double ph = s->ku * zp, by, bz;
    if (s->und_len > 0.0 && zp > s->und_len) {
        /* past the exit (reading R26): the entrance fringe mirrored about
           z' = L, which joins the last whole period in value and slope */
        double pe = s->ku * (zp - s->und_len), g = exp(-pe * pe / 2.0);
        by = s->B0 * cosh(s->ku * y) * pe * g;
        bz = s->B0 * sinh(s->ku * y) * g;
    } else if (zp >= 0.0) {
        by = s->B0 * cosh(s->ku * y) * sin(ph);
        bz = s->B0 * sinh(s->ku * y) * cos(ph);
    } else {
        double g = exp(-ph * ph / 2.0);
        by = s->B0 * cosh(s->ku * y) * ph * g;
        bz = s->B0 * sinh(s->ku * y) * g;
    }
    E[0] = -s->gamma0 * s->beta0 * ORC_C * by;
    E[1] = 0.0;
    E[2] = 0.0;
    B[0] = 0.0;
    B[1] = s->gamma0 * by;
    B[2] = bz;
}

/* ---- O7: Boris scheme, eq. (BorisScheme), for a charge q and mass m ------- */

void orc_boris(double q, double m, double dtb, double *u, const double *E, const double *B)
{
    double h = q * dtb / (2.0 * m * ORC_C);
    double t1[3] = {u[0] + h * E[0], u[1] + h * E[1], u[2] + h * E[2]};
    double alpha = q * dtb / (2.0 * m * sqrt(1.0 + t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]));
    double t2[3] = {t1[0] + alpha * (t1[1] * B[2] - t1[2] * B[1]),
                    t1[1] + alpha * (t1[2] * B[0] - t1[0] * B[2]),
                    t1[2] + alpha * (t1[0] * B[1] - t1[1] * B[0])};
    double fac = 2.0 * alpha / (1.0 + alpha * alpha * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]));
    double w[3] = {fac * B[0], fac * B[1], fac * B[2]};
    double t3[3] = {t1[0] + (t2[1] * w[2] - t2[2] * w[1]),
                    t1[1] + (t2[2] * w[0] - t2[0] * w[2]),
                    t1[2] + (t2[0] * w[1] - t2[1] * w[0])};
    u[0] = t3[0] + h * E[0];
    u[1] = t3[1] + h * E[1];
    u[2] = t3[2] + h * E[2];
}

void orc_push(orc_sim *s)
{
    double t0 = (s->step + 0.5) * s->dt;
    long lost = 0;
    int nonfinite = 0;
#pragma omp parallel for schedule(static) reduction(+ : lost) reduction(| : nonfinite)
    for (long p = 0; p < s->np; p++) {
        double *x = &s->x[3 * p], *u = &s->u[3 * p];
        s->x_old[3 * p + 0] = x[0];
        s->x_old[3 * p + 1] = x[1];
        s->x_old[3 * p + 2] = x[2];
        if (!s->alive[p]) continue;
        double Eg[3], Bg[3];
        orc_gather(s, x, Eg, Bg); /* reading R6 */
        for (int sub = 0; sub < s->N; sub++) {
            double ts = t0 + sub * s->dtb, Eu[3], Bu[3], Et[3], Bt[3];
            orc_undulator(s, x[0], x[1], x[2], ts, Eu, Bu);
            for (int a = 0; a < 3; a++) {
                Et[a] = Eg[a] + Eu[a];
                Bt[a] = Bg[a] + Bu[a];
            }
            orc_boris(s->q, s->m, s->dtb, u, Et, Bt);
            double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int a = 0; a < 3; a++) x[a] += ORC_C * s->dtb * u[a] / g;
        }
        if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(x[0]) &&
              isfinite(x[1]) && isfinite(x[2]))) {
            nonfinite = 1;
            s->alive[p] = 0;
            lost++;
            continue;
        }
        /* O8: loss (reading R17) */
        int c[3];
        double f[3];
        cell_of(s, x, c, f);
        if (!inside(s, c)) {
            s->alive[p] = 0;
            lost++;
        }
    }
    s->lost += lost;
    if (nonfinite) s->nonfinite_u = 1;
}

/* ---- O9: deposit rho^{n+3/2} and J^{n+1} ---------------------------------- */

void orc_deposit(orc_sim *s)
{
    memcpy(s->rho_prev, s->rho, sizeof(double) * s->ncell);
    memset(s->rho, 0, sizeof(double) * s->ncell);
    for (int c = 0; c < 3; c++) memset(s->J[c], 0, sizeof(double) * s->ncell);
    for (long p = 0; p < s->np; p++) {
        if (!s->alive[p]) continue;
        deposit_rho(s, s->rho, &s->x[3 * p]);
        orc_deposit_current(s, &s->x_old[3 * p], &s->x[3 * p]);
    }
}

/* ---- O10: diagnostics, one row per step ------------------------------------
   row: step, t, total charge, continuity residual, radiated power through the
   plane k = kp, field energy, kinetic energy, probe E (3), probe B (3), lost,
   non-finite flag, spare, bunching factor at harmonics 1..3, spare, power at
   the harmonics 1..3 through the plane k = kp, spare, radiated power through
   the further plates (0 where none).

   Bunching factor (the quantity <exp(j k z)> of section "Bunching factor",
   reading R21): b_h = |(1/N) sum_p exp(i h K z_p)| over the N live particles,
   z_p the rest-frame longitudinal position and K = 2 gamma0 k_u, the wave
   number of the ponderomotive phase in the frame of the undulator-averaged
   bunch (k_u = 2 pi / lambda_u in the lab). */

/* Power at the normalized frequencies nu_f of the rest-frame resonant
   frequency omega_1 = gamma0 beta0 c k_u through the power plane (reading
   R22; section "FEL-OUTPUT", normalized-frequency and its sweep).  Each step
   adds the sample at t = (s + 1/2) dt to the running DFT
   F(omega) = sum_n f(t_n) exp(-i omega t_n) dt of Ex, Ey, Bx, By at every
   plane point; after T = (number of samples) dt the mean power carried at
   omega is (2 / T^2) sum_plane Re(F_Ex conj(F_By) - F_Ey conj(F_Bx)) / mu0 dx dy,
   which for a field that is a pure tone over whole periods equals the time
   mean of the instantaneous Poynting flux.  The normalized frequency is the
   same in both frames for waves along z. */

static double omega1(const orc_sim *s)
{
    return s->gamma0 * s->beta0 * ORC_C * (2.0 * ORC_PI / s->lambda_u);
}

void orc_spectrum_sample(orc_sim *s)
{
    int lo[2], hi[2];
    for (int a = 0; a < 2; a++) interior(s, a, &lo[a], &hi[a]);
    const double t = (s->step + 0.5) * s->dt;
    const int nf = s->nfreq;
    for (int fq = 0; fq < nf; fq++) {
        const double w = s->fnu[fq] * omega1(s);
        const double cs = cos(w * t), sn = sin(w * t);
#pragma omp parallel for schedule(static)
        for (int j = lo[1]; j <= hi[1]; j++)
            for (int i = lo[0]; i <= hi[0]; i++) {
                long p = IX(s, i, j, s->kp);
                const double f[4] = {s->E[0][p], s->E[1][p], s->B[0][p], s->B[1][p]};
                double *acc = &s->spec[(((long)j * s->n[0] + i) * nf + fq) * 8];
                for (int c = 0; c < 4; c++) {
                    acc[2 * c] += f[c] * cs * s->dt;
                    acc[2 * c + 1] -= f[c] * sn * s->dt;
                }
            }
    }
    s->nspec++;
}

/* The fields of the bunch frame seen in the lab (the frame moves along +z at
   beta0 c): E_x = g (E'_x + b c B'_y), E_y = g (E'_y - b c B'_x),
   B_x = g (B'_x - b E'_y / c), B_y = g (B'_y + b E'_x / c), E_z and B_z
   unchanged (section "Lorentz Transformation").  f = (Ex, Ey, Bx, By). */
static void to_lab(const orc_sim *s, const double *f, double *lab)
{
    const double g = s->gamma0, b = s->beta0;
    lab[0] = g * (f[0] + b * ORC_C * f[3]);
    lab[1] = g * (f[1] - b * ORC_C * f[2]);
    lab[2] = g * (f[2] - b * f[1] / ORC_C);
    lab[3] = g * (f[3] + b * f[0] / ORC_C);
}

/* mean power at each frequency since the restart, in the bunch frame (rest)
   and, from the same DFT sums taken to the lab by to_lab, in the lab */
static void spectrum_power(const orc_sim *s, double *rest, double *lab)
{
    int lo[2], hi[2];
    for (int a = 0; a < 2; a++) interior(s, a, &lo[a], &hi[a]);
    const double T = s->nspec * s->dt;
    const int nf = s->nfreq;
    for (int fq = 0; fq < nf; fq++) {
        double sr = 0.0, sl = 0.0;
        for (int j = lo[1]; j <= hi[1]; j++)
            for (int i = lo[0]; i <= hi[0]; i++) {
                const double *a = &s->spec[(((long)j * s->n[0] + i) * nf + fq) * 8];
                /* a[0..1] Ex, a[2..3] Ey, a[4..5] Bx, a[6..7] By (re, im) */
                sr += (a[0] * a[6] + a[1] * a[7]) - (a[2] * a[4] + a[3] * a[5]);
                const double re[4] = {a[0], a[2], a[4], a[6]}, im[4] = {a[1], a[3], a[5], a[7]};
                double lr[4], li[4];
                to_lab(s, re, lr);
                to_lab(s, im, li);
                sl += (lr[0] * lr[3] + li[0] * li[3]) - (lr[1] * lr[2] + li[1] * li[2]);
            }
        const double k = s->nspec > 0 ? 2.0 / (T * T) / ORC_MU0 * s->d[0] * s->d[1] : 0.0;
        rest[fq] = k * sr;
        lab[fq] = k * sl;
    }
}

static void bunching(const orc_sim *s, double *b)
{
    const double K = 2.0 * s->gamma0 * (2.0 * ORC_PI / s->lambda_u);
    double re[3] = {0.0, 0.0, 0.0}, im[3] = {0.0, 0.0, 0.0};
    long n = 0;
    for (long p = 0; p < s->np; p++) {
        if (!s->alive[p]) continue;
        n++;
        for (int h = 1; h <= 3; h++) {
            re[h - 1] += cos(h * K * s->x[3 * p + 2]);
            im[h - 1] += sin(h * K * s->x[3 * p + 2]);
        }
    }
    for (int h = 0; h < 3; h++) b[h] = n > 0 ? sqrt(re[h] * re[h] + im[h] * im[h]) / (double)n : 0.0;
}

/* the flux of the lab Poynting vector of the self field (the fields of
   plane k taken to the lab by to_lab) through the plane k */
static double plane_power_lab(const orc_sim *s, int k)
{
    int lo[2], hi[2];
    for (int a = 0; a < 2; a++) interior(s, a, &lo[a], &hi[a]);
    double power = 0.0;
    for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
            long p = IX(s, i, j, k);
            const double f[4] = {s->E[0][p], s->E[1][p], s->B[0][p], s->B[1][p]};
            double l[4];
            to_lab(s, f, l);
            power += (l[0] * l[3] - l[1] * l[2]) / ORC_MU0 * s->d[0] * s->d[1];
        }
    return power;
}

/* radiated power: the flux of the Poynting vector of the self field through
   the plane k, over the interior points */
static double plane_power(const orc_sim *s, int k)
{
    int lo[2], hi[2];
    for (int a = 0; a < 2; a++) interior(s, a, &lo[a], &hi[a]);
    double power = 0.0;
    for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
            long p = IX(s, i, j, k);
            power += (s->E[0][p] * s->B[1][p] - s->E[1][p] * s->B[0][p]) / ORC_MU0 * s->d[0] * s->d[1];
        }
    return power;
}

static void diag_row(orc_sim *s, double *row, double *rest, double *lab);

void orc_diag_row(orc_sim *s, double *row)
{
    double rest[ORC_MAXF], lab[ORC_MAXF];
    diag_row(s, row, rest, lab);
}

/* the row, and the mean power at each frequency in the bunch frame (rest)
   and in the lab (lab) */
static void diag_row(orc_sim *s, double *row, double *rest, double *lab)
{
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) interior(s, a, &lo[a], &hi[a]);
    double dx = s->d[0], dy = s->d[1], dz = s->d[2], dV = dx * dy * dz;
    double charge = 0.0, rmax = 0.0, resmax = 0.0;
    for (long p = 0; p < s->ncell; p++) {
        charge += s->rho[p] * dV;
        if (fabs(s->rho[p]) > rmax) rmax = fabs(s->rho[p]);
    }
    for (int k = 1; k < s->n[2]; k++)
        for (int j = 1; j < s->n[1]; j++)
            for (int i = 1; i < s->n[0]; i++) {
                long p = IX(s, i, j, k);
                double div = (s->J[0][p] - s->J[0][IX(s, i - 1, j, k)]) / dx +
                             (s->J[1][p] - s->J[1][IX(s, i, j - 1, k)]) / dy +
                             (s->J[2][p] - s->J[2][IX(s, i, j, k - 1)]) / dz;
                double r = fabs(s->rho[p] - s->rho_prev[p] + s->dt * div);
                if (r > resmax) resmax = r;
            }
    double power = plane_power(s, s->kp);
    double wf = 0.0;
    for (int k = lo[2]; k <= hi[2]; k++)
        for (int j = lo[1]; j <= hi[1]; j++)
            for (int i = lo[0]; i <= hi[0]; i++) {
                long p = IX(s, i, j, k);
                double e2 = s->E[0][p] * s->E[0][p] + s->E[1][p] * s->E[1][p] + s->E[2][p] * s->E[2][p];
                double b2 = s->B[0][p] * s->B[0][p] + s->B[1][p] * s->B[1][p] + s->B[2][p] * s->B[2][p];
                wf += (0.5 * ORC_EPS0 * e2 + 0.5 * b2 / ORC_MU0) * dV;
            }
    double wk = 0.0;
    for (long p = 0; p < s->np; p++) {
        if (!s->alive[p]) continue;
        const double *u = &s->u[3 * p];
        wk += (sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) - 1.0) * s->m * ORC_C * ORC_C;
    }
    long pp = IX(s, s->probe[0], s->probe[1], s->probe[2]);
    row[0] = (double)s->step;
    row[1] = (s->step + 0.5) * s->dt;
    row[2] = charge;
    row[3] = rmax > 0.0 ? resmax / rmax : 0.0;
    row[4] = power;
    row[5] = wf;
    row[6] = wk;
    for (int a = 0; a < 3; a++) {
        row[7 + a] = s->E[a][pp];
        row[10 + a] = s->B[a][pp];
    }
    row[13] = (double)s->lost;
    int nf = s->nonfinite_u;
    for (int a = 2; a < 13; a++)
        if (!isfinite(row[a])) nf = 1;
    row[14] = nf;
    row[15] = 0.0;
    bunching(s, &row[16]);
    row[19] = 0.0;
    spectrum_power(s, rest, lab);
    for (int f = 0; f < 3; f++) row[20 + f] = f < s->nfreq ? rest[f] : 0.0;
    row[23] = 0.0;
    for (int e = 0; e < 3; e++) row[24 + e] = s->kp_extra[e] >= 0 ? plane_power(s, s->kp_extra[e]) : 0.0;
    /* FEL output in the lab: the lab flux through the plane and the plane's
       position along the undulator at the row's time */
    row[27] = plane_power_lab(s, s->kp);
    row[28] = s->gamma0 * (s->o[2] + s->kp * s->d[2] - s->z_e + s->beta0 * ORC_C * row[1]);
}

/* ---- O11: rotate the time levels ------------------------------------------ */

void orc_rotate(orc_sim *s)
{
    int t = s->lprev;
    s->lprev = s->lcur;
    s->lcur = s->lnext;
    s->lnext = t;
    s->step++;
}

/* one full time step in the order of the method */
void orc_step(orc_sim *s, long nsteps)
{
    for (long it = 0; it < nsteps; it++) {
        orc_field_update(s);  /* potentials at n+1, Mur faces */
        orc_vertex_fields(s); /* E, B at n+1/2 */
        orc_push(s);          /* gather, undulator, Boris, loss */
        orc_deposit(s);       /* rho^{n+3/2}, J^{n+1} */
        orc_spectrum_sample(s);
        if (s->ndiag == s->cap) {
            s->cap *= 2;
            s->diag = (double *)realloc(s->diag, sizeof(double) * ORC_NDIAG * s->cap);
            s->srow = (double *)realloc(s->srow, sizeof(double) * 2 * ORC_MAXF * s->cap);
        }
        double *sr = &s->srow[2 * ORC_MAXF * s->ndiag];
        diag_row(s, &s->diag[ORC_NDIAG * s->ndiag], sr, sr + ORC_MAXF);
        s->ndiag++;
        orc_rotate(s);
    }
}

/* ---- accessors for the Python wrapper -------------------------------------- */

/* which: 0..3 potentials at level n (after a step: the newest level),
   4..7 level n-1, 8..11 the scratch level, 12..14 J, 15 rho, 16 rho_prev,
   17..19 E, 20..22 B, 23 x, 24 u, 25 x_old, 26 diag rows */
double *orc_array(orc_sim *s, int which)
{
    if (which < 4) return s->pot[s->lcur][which];
    if (which < 8) return s->pot[s->lprev][which - 4];
    if (which < 12) return s->pot[s->lnext][which - 8];
    if (which < 15) return s->J[which - 12];
    if (which == 15) return s->rho;
    if (which == 16) return s->rho_prev;
    if (which < 20) return s->E[which - 17];
    if (which < 23) return s->B[which - 20];
    if (which == 23) return s->x;
    if (which == 24) return s->u;
    if (which == 25) return s->x_old;
    if (which == 26) return s->diag;
    if (which == 27) return s->srow;
    return NULL;
}

unsigned char *orc_alive(orc_sim *s) { return s->alive; }

long orc_info(orc_sim *s, int which)
{
    switch (which) {
    case 0: return s->np;
    case 1: return s->step;
    case 2: return s->lost;
    case 3: return s->ndiag;
    case 4: return s->ncell;
    default: return -1;
    }
}

/* threads the loops without floating-point reductions run on (1 unless
   built with OpenMP, which changes no result: those loops write disjoint
   points or particles, and every sum stays sequential) */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the step counter (the time levels the next step uses: potentials at
   n, particles at n + 1/2).  For checks that load a state taken elsewhere. */
void orc_set_step(orc_sim *s, long step) { s->step = step; }

/* derived constants: dt, dtb, A, a1, a2, a4, a6, a8, gamma0, beta0, B0, ku,
   mur-z beta0, beta1, mu0, eps0, c, e, me */
void orc_constants(const orc_sim *s, double *out)
{
    out[0] = s->dt;
    out[1] = s->dtb;
    out[2] = s->A;
    out[3] = s->a1;
    out[4] = s->a2;
    out[5] = s->a4;
    out[6] = s->a6;
    out[7] = s->a8;
    out[8] = s->gamma0;
    out[9] = s->beta0;
    out[10] = s->B0;
    out[11] = s->ku;
    out[12] = s->mur[2][0];
    out[13] = s->mur[2][1];
    out[14] = ORC_MU0;
    out[15] = ORC_EPS0;
    out[16] = ORC_C;
    out[17] = ORC_QE;
    out[18] = ORC_ME;
}
