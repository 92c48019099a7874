/* Test driver for the oracle under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Test infrastructure: built by tests/sanitize/build.py with gcc -fsanitize=address,
 * undefined into a standalone executable (no preloaded runtime), once from the FP64
 * oracle and once from its extended-precision build.  It includes the oracle's source
 * so that the executable holds one translation unit.  Every input buffer is read from
 * a raw file into an allocation of exactly the file's size, so a read past the end of
 * any array the oracle is given is a reported heap overflow.
 *
 * Modes (numbers in decimal; files are raw native-endian arrays):
 *   fields  CHARGES PTS TIMES KIND MASK OUT FLAGS
 *       or_fields over the charges (or_traj records), points ([3][n]) and times;
 *       writes OUT ([n_times][10][n]) and FLAGS (uint32 [n]); prints "status S".
 *   pair    CHARGES I X Y Z T KIND MASK
 *       or_traj_kin, or_retarded_tau and or_lw_pair of charge I; prints their
 *       statuses and values.
 *   dipole  DIPOLES OFFSETS DT STEPS POLICY MAX_VEL STRIDE PREFIX [PTS TIMES]
 *       or_dipole_run (16 doubles per dipole: origin[3], axis[3], omega0, q, m1, m2,
 *       d0, motion_amp[3], motion_omega, motion_phase; int32 offsets), writing
 *       PREFIX.d .v .E .Ed .Wabs .Wrad .hist; with PTS and TIMES also
 *       or_dipole_fields into PREFIX.field; prints the statuses.
 *   hist    HIST N_DIP JD N DT D0 TP
 *       or_hist_at; prints its status and (d, d_dot, d_ddot).
 */
#include "../../oracle/lw_oracle.c"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static void *read_file(const char *path, size_t *bytes)
{
    FILE *f = fopen(path, "rb");
    long n;
    void *p;
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        exit(2);
    }
    fseek(f, 0, SEEK_END);
    n = ftell(f);
    fseek(f, 0, SEEK_SET);
    p = malloc(n > 0 ? (size_t)n : 1);
    if (!p || (n > 0 && fread(p, 1, (size_t)n, f) != (size_t)n)) {
        fprintf(stderr, "cannot read %s\n", path);
        exit(2);
    }
    fclose(f);
    *bytes = (size_t)n;
    return p;
}

static void write_file(const char *path, const void *p, size_t bytes)
{
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot write %s\n", path);
        exit(2);
    }
    fclose(f);
}

static void *alloc(size_t bytes)
{
    void *p = malloc(bytes > 0 ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static int mode_fields(char **a)
{
    size_t bc, bp, bt;
    or_traj *ch = (or_traj *)read_file(a[0], &bc);
    double *pts = (double *)read_file(a[1], &bp);
    double *times = (double *)read_file(a[2], &bt);
    const int n_ch = (int)(bc / sizeof(or_traj));
    const int64_t n_pts = (int64_t)(bp / (3 * sizeof(double)));
    const int n_t = (int)(bt / sizeof(double));
    double *out = (double *)alloc(sizeof(double) * 10 * (size_t)n_pts * (size_t)n_t);
    uint32_t *flags = (uint32_t *)alloc(sizeof(uint32_t) * (size_t)n_pts);
    const int st = or_fields(ch, n_ch, pts, n_pts, times, n_t, atoi(a[3]), atof(a[4]), out, flags);
    printf("status %d\n", st);
    write_file(a[5], out, sizeof(double) * 10 * (size_t)n_pts * (size_t)n_t);
    write_file(a[6], flags, sizeof(uint32_t) * (size_t)n_pts);
    free(ch);
    free(pts);
    free(times);
    free(out);
    free(flags);
    return 0;
}

static int mode_pair(char **a)
{
    size_t bc;
    or_traj *ch = (or_traj *)read_file(a[0], &bc);
    const int i = atoi(a[1]);
    double x[3], r[3], v[3], acc[3], j[3], tau = 0.0, out[10];
    int it = 0, st, k;
    unsigned fl;
    const double t = atof(a[5]);
    if (i < 0 || (size_t)i >= bc / sizeof(or_traj)) {
        fprintf(stderr, "charge index out of range\n");
        return 2;
    }
    x[0] = atof(a[2]);
    x[1] = atof(a[3]);
    x[2] = atof(a[4]);
    st = or_traj_kin(&ch[i], t, r, v, acc, j);
    printf("kin %d", st);
    for (k = 0; k < 3; ++k) printf(" %.17g", r[k]);
    for (k = 0; k < 3; ++k) printf(" %.17g", v[k]);
    for (k = 0; k < 3; ++k) printf(" %.17g", acc[k]);
    for (k = 0; k < 3; ++k) printf(" %.17g", j[k]);
    st = or_retarded_tau(&ch[i], x, t, &tau, &it);
    printf("\ntau %d %.17g %d\n", st, tau, it);
    fl = or_lw_pair(&ch[i], x, t, atoi(a[6]), atof(a[7]), out);
    printf("pair %u", fl);
    for (k = 0; k < 10; ++k) printf(" %.17g", fl ? 0.0 : out[k]);
    printf("\n");
    free(ch);
    return 0;
}

static int mode_dipole(char **a, int n_args)
{
    size_t bd, bo;
    double *rec = (double *)read_file(a[0], &bd);
    int32_t *off = (int32_t *)read_file(a[1], &bo);
    const int n = (int)(bd / (16 * sizeof(double)));
    const int n_inst = (int)(bo / sizeof(int32_t)) - 1;
    const double dt = atof(a[2]);
    const int64_t steps = atoll(a[3]);
    const int policy = atoi(a[4]);
    const double max_vel = atof(a[5]);
    const int64_t stride = atoll(a[6]);
    const char *prefix = a[7];
    const int64_t n_out = steps / stride + 1;
    const size_t ob = sizeof(double) * (size_t)n_out * (size_t)n;
    const size_t hb = sizeof(double) * (size_t)(steps + 1) * (size_t)n * 3;
    double *origin = (double *)alloc(sizeof(double) * 3 * n), *axis = (double *)alloc(sizeof(double) * 3 * n);
    double *omega0 = (double *)alloc(sizeof(double) * n), *q = (double *)alloc(sizeof(double) * n);
    double *m1 = (double *)alloc(sizeof(double) * n), *m2 = (double *)alloc(sizeof(double) * n);
    double *d0 = (double *)alloc(sizeof(double) * n), *mamp = (double *)alloc(sizeof(double) * 3 * n);
    double *mom = (double *)alloc(sizeof(double) * n), *mph = (double *)alloc(sizeof(double) * n);
    double *od = (double *)alloc(ob), *ov = (double *)alloc(ob), *oE = (double *)alloc(ob);
    double *oEd = (double *)alloc(ob), *oWa = (double *)alloc(ob), *oWr = (double *)alloc(ob);
    double *hist = (double *)alloc(hb);
    int i, k, moving = 0, st;
    char path[4096];
    for (i = 0; i < n; ++i) {
        const double *r = rec + 16 * i;
        for (k = 0; k < 3; ++k) {
            origin[3 * i + k] = r[k];
            axis[3 * i + k] = r[3 + k];
            mamp[3 * i + k] = r[11 + k];
            moving |= r[11 + k] != 0.0;
        }
        omega0[i] = r[6];
        q[i] = r[7];
        m1[i] = r[8];
        m2[i] = r[9];
        d0[i] = r[10];
        mom[i] = r[14];
        mph[i] = r[15];
    }
    st = or_dipole_run(n, origin, axis, omega0, q, m1, m2, d0, moving ? mamp : NULL, moving ? mom : NULL,
                       moving ? mph : NULL, n_inst, off, dt, steps, policy, max_vel, stride, od, ov, oE, oEd, oWa,
                       oWr, hist);
    printf("run %d\n", st);
    if (st == OR_OK) {
        static const char *ext[7] = {"d", "v", "E", "Ed", "Wabs", "Wrad", "hist"};
        double *arr[7];
        arr[0] = od; arr[1] = ov; arr[2] = oE; arr[3] = oEd; arr[4] = oWa; arr[5] = oWr; arr[6] = hist;
        for (k = 0; k < 7; ++k) {
            snprintf(path, sizeof path, "%s.%s", prefix, ext[k]);
            write_file(path, arr[k], k == 6 ? hb : ob);
        }
        if (n_args >= 10) {
            size_t bp, bt;
            double *pts = (double *)read_file(a[8], &bp);
            double *times = (double *)read_file(a[9], &bt);
            const int64_t n_pts = (int64_t)(bp / (3 * sizeof(double)));
            const int n_t = (int)(bt / sizeof(double));
            double *E = (double *)alloc(sizeof(double) * 3 * (size_t)n_pts * (size_t)n_t);
            st = or_dipole_fields(n, origin, axis, q, m1, m2, d0, moving ? mamp : NULL, moving ? mom : NULL,
                                  moving ? mph : NULL, dt, steps, hist, pts, n_pts, times, n_t, E);
            printf("fields %d\n", st);
            snprintf(path, sizeof path, "%s.field", prefix);
            write_file(path, E, sizeof(double) * 3 * (size_t)n_pts * (size_t)n_t);
            free(pts);
            free(times);
            free(E);
        }
    }
    free(rec); free(off); free(origin); free(axis); free(omega0); free(q); free(m1); free(m2); free(d0);
    free(mamp); free(mom); free(mph); free(od); free(ov); free(oE); free(oEd); free(oWa); free(oWr); free(hist);
    return 0;
}

static int mode_hist(char **a)
{
    size_t bh, bd;
    double *hist = (double *)read_file(a[0], &bh);
    double *d0 = (double *)read_file(a[5], &bd);
    double out[3] = {0.0, 0.0, 0.0};
    const int st = or_hist_at(hist, atoi(a[1]), atoi(a[2]), atoll(a[3]), atof(a[4]), d0, atof(a[6]), out);
    printf("hist %d %.17g %.17g %.17g\n", st, out[0], out[1], out[2]);
    free(hist);
    free(d0);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc >= 2 && !strcmp(argv[1], "digits")) {
        printf("digits %d\n", or_real_digits());
        return 0;
    }
    if (argc == 9 && !strcmp(argv[1], "fields")) return mode_fields(argv + 2);
    if (argc == 10 && !strcmp(argv[1], "pair")) return mode_pair(argv + 2);
    if ((argc == 10 || argc == 12) && !strcmp(argv[1], "dipole")) return mode_dipole(argv + 2, argc - 2);
    if (argc == 9 && !strcmp(argv[1], "hist")) return mode_hist(argv + 2);
    fprintf(stderr, "usage: see the header of oracle_driver.c\n");
    return 2;
}
