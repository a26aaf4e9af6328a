/* Test driver: runs the oracle over a workload read from a file, for a build
 * of the oracle with AddressSanitizer and UndefinedBehaviorSanitizer (and
 * its own asserts, e.g. the one-cell move of a particle in a step that the
 * charge-conserving deposit relies on).  Test infrastructure only.
 *
 * Input (doubles): n[3], d[3], origin[3], courant, nsfd_A, substeps,
 * space_charge, bc[3], lambda_u, K, gamma, z_entrance, q, m, np, steps,
 * probe[3], kp, undulator length, number of normalized frequencies (<= 32),
 * extra plates k1..k3 (-1: none), then nu[nfreq], positions [np][3] and
 * momenta [np][3].  Output on stdout: steps run, diagnostic rows, lost
 * particles, and the sum of the last diagnostic row (a checksum).  Exit
 * status 0 on success. */
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_sim orc_sim;
orc_sim *orc_create(const int n[3], const double d[3], const double origin[3], double courant,
                    double nsfd_A, int substeps, int space_charge, const int bc[3],
                    double lambda_u, double K, double gamma_beam, double z_e);
void orc_destroy(orc_sim *s);
void orc_config_diag(orc_sim *s, int pi, int pj, int pk, int kp);
void orc_set_spectrum(orc_sim *s, const double *nu, int nfreq);
void orc_set_undulator_length(orc_sim *s, double length);
void orc_config_extra_planes(orc_sim *s, int k1, int k2, int k3);
int orc_set_particles(orc_sim *s, long np, const double *x, const double *u, double q, double m);
void orc_step(orc_sim *s, long nsteps);
double *orc_array(orc_sim *s, int which);
long orc_info(orc_sim *s, int which);

#define NHEAD 33

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 3;
    double h[NHEAD];
    if (fread(h, sizeof(double), NHEAD, f) != NHEAD) return 4;
    const int n[3] = {(int)h[0], (int)h[1], (int)h[2]};
    const int bc[3] = {(int)h[13], (int)h[14], (int)h[15]};
    const long np = (long)h[22], steps = (long)h[23];
    const int nfreq = (int)h[29];
    if (nfreq < 0 || nfreq > 32 || np < 0) return 5;
    double *nu = malloc(sizeof(double) * (nfreq > 0 ? nfreq : 1));
    double *x = malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    double *u = malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    if ((long)fread(nu, sizeof(double), nfreq, f) != nfreq) return 6;
    if ((long)fread(x, sizeof(double), 3 * np, f) != 3 * np) return 7;
    if ((long)fread(u, sizeof(double), 3 * np, f) != 3 * np) return 8;
    fclose(f);
    orc_sim *s = orc_create(n, h + 3, h + 6, h[9], h[10], (int)h[11], (int)h[12], bc, h[16], h[17],
                            h[18], h[19]);
    orc_config_diag(s, (int)h[24], (int)h[25], (int)h[26], (int)h[27]);
    orc_set_undulator_length(s, h[28]);
    orc_config_extra_planes(s, (int)h[30], (int)h[31], (int)h[32]);
    if (nfreq > 0) orc_set_spectrum(s, nu, nfreq);
    orc_set_particles(s, np, x, u, h[20], h[21]);
    orc_step(s, steps);
    const double *diag = orc_array(s, 26);
    double sum = 0.0;
    const long rows = orc_info(s, 3);
    if (diag && rows > 0)
        for (int c = 0; c < 29; c++) sum += diag[(rows - 1) * 29 + c];
    printf("%ld %ld %ld %.17g\n", orc_info(s, 1), rows, orc_info(s, 2), sum);
    orc_destroy(s);
    free(nu);
    free(x);
    free(u);
    return 0;
}
