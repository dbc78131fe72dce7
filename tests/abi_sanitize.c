/*
 * Host-side driver for the AddressSanitizer / UndefinedBehaviorSanitizer run
 * of the C ABI's argument validation (tests/test_host_sanitizers.py builds the
 * library's host code with both sanitizers and runs this program; no GPU is
 * used).  Every input array is allocated with exactly the size the header
 * states, so a read past its end is reported by AddressSanitizer.  Each call
 * must return the documented status: EINVAL for bad arguments, and for valid
 * arguments EDEVICE when no device is present (or OK, then the problem is
 * destroyed again).  Prints "abi_sanitize: <checks> checks passed" on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "xfft.h"

static int g_checks = 0, g_fail = 0;

static void expect(int got, int want, const char *what) {
    ++g_checks;
    if (got != want) {
        ++g_fail;
        fprintf(stderr, "FAIL %s: got %d, want %d\n", what, got, want);
    }
}

typedef struct {
    int32_t n[3];
    double len[3];
    double *L;
    int32_t *ph;
    int32_t nphase;
    double *lame;
} Case;

static Case make_case(int n0, int n1, int n2, int nphase) {
    Case c;
    c.n[0] = n0; c.n[1] = n1; c.n[2] = n2;
    c.len[0] = n0; c.len[1] = n1; c.len[2] = n2;
    const size_t N = (size_t)n0 * n1 * n2;
    c.L = (double *)malloc(sizeof(double) * N);
    c.ph = (int32_t *)malloc(sizeof(int32_t) * N);
    c.nphase = nphase;
    c.lame = (double *)malloc(sizeof(double) * 2 * nphase);
    for (size_t q = 0; q < N; ++q) {
        const int i = (int)(q % n0), j = (int)((q / n0) % n1), k = (int)(q / ((size_t)n0 * n1));
        const double dx = i - 0.5 * n0 + 0.31, dy = j - 0.5 * n1 - 0.17, dz = k - 0.5 * n2 + 0.23;
        c.L[q] = sqrt(dx * dx + dy * dy + dz * dz) - 0.3 * n0;
        c.ph[q] = c.L[q] < 0.0 ? (nphase > 1 ? 1 : 0) : 0;
    }
    for (int p = 0; p < nphase; ++p) {
        c.lame[2 * p] = 0.5 + p;
        c.lame[2 * p + 1] = 0.4 + 0.5 * p;
    }
    return c;
}

static void free_case(Case *c) {
    free(c->L);
    free(c->ph);
    free(c->lame);
}

/* valid arguments: EDEVICE without a device, OK with one */
static void expect_valid(const Case *c, const xfft_options *opt, const char *what) {
    xfft_problem *p = (xfft_problem *)0x1;
    const int rc = xfft_setup(c->n, c->len, c->L, c->ph, c->nphase, c->lame, opt, &p);
    ++g_checks;
    if (rc == XFFT_OK) {
        xfft_destroy(p);
    } else if (rc != XFFT_EDEVICE || p != NULL) {
        ++g_fail;
        fprintf(stderr, "FAIL %s: got %d\n", what, rc);
    }
}

static void expect_setup(const Case *c, const xfft_options *opt, int want, const char *what) {
    xfft_problem *p = (xfft_problem *)0x1;
    const int rc = xfft_setup(c->n, c->len, c->L, c->ph, c->nphase, c->lame, opt, &p);
    expect(rc, want, what);
    ++g_checks;
    if (p != NULL) {
        ++g_fail;
        fprintf(stderr, "FAIL %s: *out not cleared\n", what);
    }
}

int main(void) {
    /* defaults, strerror, destroy(NULL) */
    xfft_default_options(NULL);
    xfft_options def;
    memset(&def, 0xff, sizeof(def));
    xfft_default_options(&def);
    expect(def.precision, XFFT_FP64, "default precision");
    expect(def.batch, 1, "default batch");
    for (int code = -6; code <= 3; ++code) {
        const char *s = xfft_strerror(code);
        ++g_checks;
        if (!s || !s[0]) { ++g_fail; fprintf(stderr, "FAIL strerror(%d)\n", code); }
    }
    xfft_destroy(NULL);

    Case c = make_case(16, 12, 8, 2);
    expect_valid(&c, NULL, "valid 16x12x8");
    expect_valid(&c, &def, "valid 16x12x8 with explicit defaults");

    /* null pointers */
    expect(xfft_setup(c.n, c.len, c.L, c.ph, c.nphase, c.lame, NULL, NULL), XFFT_EINVAL, "out NULL");
    {
        xfft_problem *p = (xfft_problem *)0x1;
        expect(xfft_setup(NULL, c.len, c.L, c.ph, c.nphase, c.lame, NULL, &p), XFFT_EINVAL, "n NULL");
        expect(xfft_setup(c.n, NULL, c.L, c.ph, c.nphase, c.lame, NULL, &p), XFFT_EINVAL, "len NULL");
        expect(xfft_setup(c.n, c.len, NULL, c.ph, c.nphase, c.lame, NULL, &p), XFFT_EINVAL, "levelset NULL");
        expect(xfft_setup(c.n, c.len, c.L, NULL, c.nphase, c.lame, NULL, &p), XFFT_EINVAL, "phase NULL");
        expect(xfft_setup(c.n, c.len, c.L, c.ph, c.nphase, NULL, NULL, &p), XFFT_EINVAL, "lame NULL");
        expect(xfft_setup(c.n, c.len, c.L, c.ph, 0, c.lame, NULL, &p), XFFT_EINVAL, "nphase 0");
    }

    /* grid sizes: odd, too small, a factor 5, beyond the FFT limits; the arrays
       are sized for the claimed grid so that validation reads stay in bounds */
    {
        const int bad[][3] = {{15, 12, 8}, {2, 12, 8}, {16, 10, 8}, {16, 12, 7}, {16, 12, 1536}, {16, 12, 8192}};
        for (size_t k = 0; k < sizeof(bad) / sizeof(bad[0]); ++k) {
            Case b = make_case(bad[k][0], bad[k][1], bad[k][2], 2);
            char what[64];
            snprintf(what, sizeof(what), "grid %dx%dx%d", bad[k][0], bad[k][1], bad[k][2]);
            expect_setup(&b, NULL, XFFT_EINVAL, what);
            free_case(&b);
        }
    }
    /* cell lengths */
    {
        const double keep[3] = {c.len[0], c.len[1], c.len[2]};
        c.len[1] = 0.0;
        expect_setup(&c, NULL, XFFT_EINVAL, "len 0");
        c.len[1] = -12.0;
        expect_setup(&c, NULL, XFFT_EINVAL, "len < 0");
        c.len[1] = NAN;
        expect_setup(&c, NULL, XFFT_EINVAL, "len NaN");
        c.len[1] = 13.0;
        expect_setup(&c, NULL, XFFT_EINVAL, "non-cubic voxels");
        memcpy(c.len, keep, sizeof(keep));
    }
    /* moduli */
    {
        const double keep[4] = {c.lame[0], c.lame[1], c.lame[2], c.lame[3]};
        c.lame[3] = 0.0;
        expect_setup(&c, NULL, XFFT_EINVAL, "mu 0");
        c.lame[3] = keep[3];
        c.lame[2] = -1.0;
        expect_setup(&c, NULL, XFFT_EINVAL, "3 lambda + 2 mu <= 0");
        c.lame[2] = INFINITY;
        expect_setup(&c, NULL, XFFT_EINVAL, "lambda inf");
        memcpy(c.lame, keep, sizeof(keep));
    }
    /* level set and labels: bad value in the last entry (the scan must reach it) */
    {
        const size_t N = (size_t)c.n[0] * c.n[1] * c.n[2];
        const double lk = c.L[N - 1];
        c.L[N - 1] = NAN;
        expect_setup(&c, NULL, XFFT_EINVAL, "level set NaN");
        c.L[N - 1] = lk;
        const int32_t pk = c.ph[N - 1];
        c.ph[N - 1] = c.nphase;
        expect_setup(&c, NULL, XFFT_EINVAL, "phase == nphase");
        c.ph[N - 1] = -1;
        expect_setup(&c, NULL, XFFT_EINVAL, "phase < 0");
        c.ph[N - 1] = pk;
    }
    /* options */
    {
        xfft_options o;
#define BAD_OPT(field, value)                                           \
    do {                                                                \
        xfft_default_options(&o);                                       \
        o.field = value;                                                \
        expect_setup(&c, &o, XFFT_EINVAL, "option " #field " " #value); \
    } while (0)
        BAD_OPT(rtol, 0.0);
        BAD_OPT(rtol, NAN);
        BAD_OPT(maxit, 0);
        BAD_OPT(precision, XFFT_FP32);
        BAD_OPT(precision, 7);
        BAD_OPT(snap_eps, -1.0);
        BAD_OPT(d0_scale, 0.0);
        BAD_OPT(inner_rtol, 1.0);
        BAD_OPT(inner_rtol, 0.0);
        BAD_OPT(scheme, -1);
        BAD_OPT(scheme, 4);
        BAD_OPT(discretization, 2);
        BAD_OPT(voxel_matrices, 2);
        BAD_OPT(voxel_matrices, -2);
        BAD_OPT(warm_start, 2);
        BAD_OPT(warm_start, -1);
        BAD_OPT(fft_variant, 4);
        BAD_OPT(fft_variant, -2);
        xfft_default_options(&o);
        o.scheme = XFFT_NLCG;
        o.precision = XFFT_MIXED;
        expect_setup(&c, &o, XFFT_EINVAL, "nonlinear CG with mixed precision");
        xfft_default_options(&o);
        o.scheme = XFFT_BB;
        expect_valid(&c, &o, "Barzilai-Borwein FP64");
        o.discretization = XFFT_P1;
        expect_valid(&c, &o, "P1 discretisation");
        xfft_default_options(&o);
        o.warm_start = 1;
        expect_valid(&c, &o, "warm start");
        xfft_default_options(&o);
        o.fft_variant = 3;
        expect_valid(&c, &o, "fixed FFT variant");
#undef BAD_OPT
    }

    /* every other entry point with a NULL problem */
    {
        double buf[64];
        int64_t info[8];
        int32_t cnt[11];
        memset(buf, 0, sizeof(buf));
        expect(xfft_set_lame(NULL, c.lame), XFFT_EINVAL, "set_lame NULL");
        expect(xfft_solve(NULL, 1, buf, NULL, NULL, NULL, NULL, NULL), XFFT_EINVAL, "solve NULL");
        expect(xfft_solve_device(NULL, 1, buf, NULL, NULL, NULL, NULL), XFFT_EINVAL, "solve_device NULL");
        expect(xfft_grad_lame(NULL, buf, buf, NULL), XFFT_EINVAL, "grad_lame NULL");
        expect(xfft_batch_solve(NULL, 1, buf, NULL), XFFT_EINVAL, "batch_solve NULL");
        expect(xfft_batch_solve(NULL, 0, buf, NULL), XFFT_EINVAL, "batch_solve empty");
        expect(xfft_apply_operator(NULL, XFFT_FP64, buf, NULL, buf, NULL), XFFT_EINVAL, "apply_operator NULL");
        expect(xfft_apply_precond(NULL, XFFT_FP64, buf, buf, NULL), XFFT_EINVAL, "apply_precond NULL");
        expect(xfft_voxel_stress(NULL, buf, NULL, buf), XFFT_EINVAL, "voxel_stress NULL");
        expect(xfft_apply_operator_noalloc(NULL, buf, NULL, buf, NULL, NULL), XFFT_EINVAL, "noalloc NULL");
        expect(xfft_get_layout(NULL, info, NULL, NULL), XFFT_EINVAL, "get_layout NULL");
        expect(xfft_profile(NULL, XFFT_FP32, 6, 1, buf, cnt), XFFT_EINVAL, "profile NULL");
        expect(xfft_profile_begin(NULL), XFFT_EINVAL, "profile_begin NULL");
        expect(xfft_profile_end(NULL, buf, cnt), XFFT_EINVAL, "profile_end NULL");
    }

    /* a larger valid grid: the full validation scan over N = 48^3 entries */
    {
        Case b = make_case(48, 48, 48, 3);
        expect_valid(&b, NULL, "valid 48^3");
        free_case(&b);
    }
    free_case(&c);

    if (g_fail) {
        fprintf(stderr, "abi_sanitize: %d of %d checks failed\n", g_fail, g_checks);
        return 1;
    }
    printf("abi_sanitize: %d checks passed\n", g_checks);
    return 0;
}
