/* Runs the CPU oracle on a case read from a binary file, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure).
 *
 * Input file: int64 n, int32 dim, int32 nsteps, double t, the parameter
 * block (its in-memory bytes), then x (n dim), u (n dim), phi (n),
 * mass (n), kind (n bytes), normal (n dim).  Output file: acc (n dim),
 * dphi (n), nnb (n int32) of one right-hand side at t, then x, u, phi after
 * nsteps steps from t. */
#include <stdio.h>

#include "../../oracle/wbsph_oracle.c"

static int rd(FILE *f, void *p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; }
static int wr(FILE *f, const void *p, size_t bytes) { return fwrite(p, 1, bytes, f) == bytes; }

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int64_t n;
    int32_t dim, nsteps;
    double t;
    orc_params p;
    if (!rd(in, &n, 8) || !rd(in, &dim, 4) || !rd(in, &nsteps, 4) || !rd(in, &t, 8) || !rd(in, &p, sizeof p))
        return 3;
    size_t nv = (size_t)n * (size_t)dim;
    double *x = malloc(8 * nv), *u = malloc(8 * nv), *phi = malloc(8 * (size_t)n), *m = malloc(8 * (size_t)n);
    double *nrm = malloc(8 * nv);
    uint8_t *kind = malloc((size_t)n);
    if (!rd(in, x, 8 * nv) || !rd(in, u, 8 * nv) || !rd(in, phi, 8 * (size_t)n) || !rd(in, m, 8 * (size_t)n) ||
        !rd(in, kind, (size_t)n) || !rd(in, nrm, 8 * nv))
        return 3;
    fclose(in);
    orc_rates r;
    if (alloc_rates(&r, n, dim) != ORC_OK) return 4;
    int st = orc_eval_rates(&p, n, x, u, phi, m, kind, nrm, t, 1, NULL, &r, NULL);
    if (st != ORC_OK) return 10 - st;
    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    if (!wr(out, r.acc, 8 * nv) || !wr(out, r.dphi, 8 * (size_t)n) || !wr(out, r.nnb, 4 * (size_t)n)) return 5;
    double dtl = 0.0;
    st = orc_step(&p, n, x, u, phi, m, kind, nrm, &t, nsteps, 0.0, 1, &dtl, NULL);
    if (st != ORC_OK) return 20 - st;
    if (!wr(out, x, 8 * nv) || !wr(out, u, 8 * nv) || !wr(out, phi, 8 * (size_t)n)) return 5;
    fclose(out);
    free_rates(&r);
    free(x); free(u); free(phi); free(m); free(nrm); free(kind);
    return 0;
}
