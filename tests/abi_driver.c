/* A plain C caller of the library: no Python, no PyTorch (hipMalloc and a
 * stream the library creates).  Reads a workload from a binary file, runs
 * it and writes the diagnostic rows and A_x.  Input, all doubles: n[3],
 * d[3], origin[3], courant, nsfd_A, substeps, space_charge, bc[3],
 * lambda_u, K, gamma, z_entrance, q, m, np, steps, probe[3], kp, the
 * undulator length, a spare value, then the positions [np][3] and momenta
 * [np][3].  Output: int64 row count, the rows
 * (mithra_diag_row), then A_x (n[0] n[1] n[2] doubles). */
#include <stdio.h>
#include <stdlib.h>

#include "mithra.h"

static int check(mithra_status st, const char *what)
{
    if (st != MITHRA_OK) {
        fprintf(stderr, "%s: status %d: %s\n", what, (int)st, mithra_last_error());
        return 1;
    }
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    double h[30];
    if (fread(h, sizeof(double), 30, in) != 30) return 2;
    mithra_mesh mesh;
    mithra_undulator und;
    for (int a = 0; a < 3; ++a) {
        mesh.n[a] = (int32_t)h[a];
        mesh.d[a] = h[3 + a];
        mesh.origin[a] = h[6 + a];
        mesh.bc[a] = (int32_t)h[13 + a];
    }
    mesh.courant = h[9];
    mesh.nsfd_A = h[10];
    mesh.substeps = (int32_t)h[11];
    mesh.space_charge = (int32_t)h[12];
    und.lambda_u = h[16];
    und.K = h[17];
    und.gamma_beam = h[18];
    und.z_entrance = h[19];
    und.length = h[28];
    const double q = h[20], m = h[21];
    const int64_t np = (int64_t)h[22], steps = (int64_t)h[23];
    double *pos = malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    double *u = malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    if (fread(pos, sizeof(double), 3 * np, in) != (size_t)(3 * np)) return 2;
    if (fread(u, sizeof(double), 3 * np, in) != (size_t)(3 * np)) return 2;
    fclose(in);

    mithra_sim *sim = NULL;
    if (check(mithra_create(&mesh, &und, MITHRA_F64, NULL, &sim), "create")) return 1;
    if (check(mithra_set_particles(sim, np, pos, u, q, m), "set_particles")) return 1;
    mithra_diag_cfg cfg = {{(int32_t)h[24], (int32_t)h[25], (int32_t)h[26]}, (int32_t)h[27], 1, 4096, 0,
                           {-1, -1, -1}};
    if (check(mithra_config_diag(sim, &cfg), "config_diag")) return 1;
    if (check(mithra_run(sim, steps), "run")) return 1;
    if (check(mithra_sync(sim), "sync")) return 1;
    mithra_diag_row *rows = malloc(sizeof(mithra_diag_row) * (size_t)steps);
    int64_t nrows = 0;
    if (check(mithra_get_diag(sim, rows, steps, &nrows), "get_diag")) return 1;
    const size_t ncell = (size_t)mesh.n[0] * mesh.n[1] * mesh.n[2];
    double *ax = malloc(sizeof(double) * ncell);
    if (check(mithra_get_field(sim, MITHRA_AX, ax), "get_field")) return 1;
    mithra_destroy(sim);
    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    fwrite(&nrows, sizeof nrows, 1, out);
    fwrite(rows, sizeof(mithra_diag_row), (size_t)nrows, out);
    fwrite(ax, sizeof(double), ncell, out);
    fclose(out);
    free(pos);
    free(u);
    free(rows);
    free(ax);
    return 0;
}
