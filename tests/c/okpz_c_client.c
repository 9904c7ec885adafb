/*
 * A plain C99 client of the okpz C ABI (include/okpz.h), with no Python in
 * between.  Built by the tests with gcc against libokpz.so.
 *
 *   okpz_c_client host           host-only calls: geometry, required bytes and
 *                                argument checks that fail before any device
 *                                call; prints "host ok"
 *   okpz_c_client run L p q seed t
 *                                a flat L x L lattice swept to MCS t: prints
 *                                "width <t> <sum_h> <sum_h2> <H0>", the axis
 *                                spectrum at n = 1, 2 and a checkpoint round
 *                                trip that must continue identically
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "okpz.h"

#define CHECK(call)                                                                   \
    do {                                                                              \
        int rc_ = (call);                                                             \
        if (rc_ != OKPZ_OK) {                                                         \
            fprintf(stderr, "%s failed: %d (%s)\n", #call, rc_, okpz_last_error());  \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

static int host_checks(void)
{
    int32_t Bx, By, C;
    CHECK(okpz_geometry(320, 192, &Bx, &By, &C));
    if (Bx != 64 || By != 64 || C != 8) return fprintf(stderr, "geometry %d %d %d\n", Bx, By, C), 1;
    CHECK(okpz_geometry((int64_t)1 << 17, 96, &Bx, &By, &C));
    if (Bx != 256 || By != 32 || C != 8) return fprintf(stderr, "geometry %d %d %d\n", Bx, By, C), 1;
    if (okpz_geometry(33, 32, &Bx, &By, &C) != OKPZ_EINVAL) return fprintf(stderr, "33 accepted\n"), 1;
    if (okpz_required_bytes(33, 32) != 0) return fprintf(stderr, "required bytes of 33\n"), 1;
    /* two copies of 2 bits per site plus a little scratch */
    size_t need = okpz_required_bytes(1024, 1024);
    if (need < 2 * 1024 * 1024 / 4 || need > 2 * 1024 * 1024 / 4 + (1 << 20))
        return fprintf(stderr, "required bytes %zu\n", need), 1;
    okpz_sim *s = (okpz_sim *)1;
    if (okpz_init(&s, 64, 64, 1.5, 0.0, 1) != OKPZ_EINVAL || s != NULL)
        return fprintf(stderr, "p = 1.5 accepted\n"), 1;
    if (strlen(okpz_last_error()) == 0) return fprintf(stderr, "no message\n"), 1;
    printf("host ok\n");
    return 0;
}

static int run(int64_t L, double p, double q, uint64_t seed, int64_t t)
{
    okpz_sim *s = NULL;
    CHECK(okpz_init(&s, L, L, p, q, seed));
    int64_t s1, s2, h0;
    CHECK(okpz_width(s, t / 2, &s1, &s2));
    size_t bytes = 0;
    CHECK(okpz_save(s, NULL, &bytes));
    void *ck = malloc(bytes);
    if (!ck) return 1;
    CHECK(okpz_save(s, ck, &bytes));
    CHECK(okpz_width(s, t, &s1, &s2));
    CHECK(okpz_h0(s, &h0));
    printf("width %lld %lld %lld %lld\n", (long long)t, (long long)s1, (long long)s2, (long long)h0);

    double *sx = malloc(sizeof(double) * (size_t)(L / 2 + 1));
    double *sy = malloc(sizeof(double) * (size_t)(L / 2 + 1));
    if (!sx || !sy) return 1;
    CHECK(okpz_psd(s, sx, sy));
    printf("psd %.17g %.17g %.17g %.17g\n", sx[1], sy[1], sx[2], sy[2]);

    okpz_sim *r = NULL;
    CHECK(okpz_load(&r, ck, bytes));
    int64_t r1, r2, rh;
    CHECK(okpz_width(r, t, &r1, &r2));
    CHECK(okpz_h0(r, &rh));
    if (r1 != s1 || r2 != s2 || rh != h0) return fprintf(stderr, "restored run differs\n"), 1;
    printf("restore ok\n");
    CHECK(okpz_free(r));
    CHECK(okpz_free(s));
    free(ck);
    free(sx);
    free(sy);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc >= 2 && strcmp(argv[1], "host") == 0) return host_checks();
    if (argc == 7 && strcmp(argv[1], "run") == 0)
        return run(atoll(argv[2]), atof(argv[3]), atof(argv[4]), strtoull(argv[5], NULL, 10),
                   atoll(argv[6]));
    fprintf(stderr, "usage: %s host | run L p q seed t\n", argv[0]);
    return 2;
}
