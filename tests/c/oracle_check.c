/* Sanitizer driver for the oracle (oracle/okpz_oracle.c), built together with
 * it under AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py.  Runs every entry point on small lattices of the
 * shapes the tests use and checks the model's invariants on the way:
 * single-valued heights (zero row and column slope sums), S1 - N/2 =
 * 2 (attachments - detachments) from the flat state, and agreement of the
 * window sweep with the whole-lattice sweep.  Prints "oracle ok". */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void or_flat(uint8_t *lat, int64_t Lx, int64_t Ly);
uint64_t or_threshold(double prob);
int or_geometry(int64_t Lx, int64_t Ly, int32_t *Bx, int32_t *By, int32_t *C);
int or_sweep(uint8_t *lat, int64_t Lx, int64_t Ly, uint64_t Tp, uint64_t Tq, uint64_t seed,
             uint32_t s, int64_t *H0, int64_t *n_att, int64_t *n_det, int check, int delayed);
void or_rsu_sweep(uint8_t *lat, int64_t Lx, int64_t Ly, uint64_t Tp, uint64_t Tq, uint64_t seed,
                  uint64_t t, int64_t *H0, int64_t *n_att, int64_t *n_det);
void or_heights(const uint8_t *lat, int64_t Lx, int64_t Ly, int64_t H0, int64_t *h);
int or_width(const uint8_t *lat, int64_t Lx, int64_t Ly, int64_t H0, int64_t *S1, int64_t *S2);
int or_ensemble_at(int64_t Lx, int64_t Ly, double p, double q, uint64_t seed0, int64_t R,
                   const int64_t *times, int64_t ntimes, int kind, int64_t *out);
int or_window_sweep(uint8_t *win, int64_t Wx, int64_t Wy, int64_t wx0, int64_t wy0, int64_t Lx,
                    int64_t Ly, uint64_t Tp, uint64_t Tq, uint64_t seed, uint32_t s,
                    int64_t *vx0, int64_t *vy0, int64_t *vx1, int64_t *vy1, int64_t *H0,
                    int delayed);

static int fails = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                                      \
        }                                                                 \
    } while (0)

static void check_single_valued(const uint8_t *lat, int64_t Lx, int64_t Ly)
{
    for (int64_t y = 0; y < Ly; ++y) {
        int64_t s = 0;
        for (int64_t x = 0; x < Lx; ++x) s += (lat[y * Lx + x] & 1) ? 1 : -1;
        CHECK(s == 0);
    }
    for (int64_t x = 0; x < Lx; ++x) {
        int64_t s = 0;
        for (int64_t y = 0; y < Ly; ++y) s += (lat[y * Lx + x] & 2) ? 1 : -1;
        CHECK(s == 0);
    }
}

static void run_shape(int64_t Lx, int64_t Ly, double p, double q, int delayed, int rsu)
{
    int32_t Bx, By, C;
    CHECK(or_geometry(Lx, Ly, &Bx, &By, &C) == 0);
    if (delayed && C < 2) return;
    uint8_t *lat = malloc((size_t)(Lx * Ly));
    int64_t *h = malloc((size_t)(Lx * Ly) * sizeof(int64_t));
    or_flat(lat, Lx, Ly);
    int64_t H0 = 0, att = 0, det = 0, S1, S2;
    const uint64_t Tp = or_threshold(p), Tq = or_threshold(q);
    for (uint32_t s = 0; s < 6; ++s) {
        if (rsu) or_rsu_sweep(lat, Lx, Ly, Tp, Tq, 11, s, &H0, &att, &det);
        else CHECK(or_sweep(lat, Lx, Ly, Tp, Tq, 11, s, &H0, &att, &det, 1, delayed) == 0);
        check_single_valued(lat, Lx, Ly);
    }
    CHECK(or_width(lat, Lx, Ly, H0, &S1, &S2) == 0);
    CHECK(S1 - Lx * Ly / 2 == 2 * (att - det));
    or_heights(lat, Lx, Ly, H0, h);
    CHECK(h[0] == H0);
    free(h);
    free(lat);
}

int main(void)
{
    static const int64_t shapes[][2] = {{4, 4}, {8, 8}, {12, 20}, {32, 32}, {96, 64},
                                        {64, 160}, {256, 256}, {320, 192}};
    for (size_t i = 0; i < sizeof shapes / sizeof shapes[0]; ++i)
        for (int kind = 0; kind < 3; ++kind) {
            run_shape(shapes[i][0], shapes[i][1], 0.95, 0.05, kind == 1, kind == 2);
            run_shape(shapes[i][0], shapes[i][1], 1.0, 0.0, kind == 1, kind == 2);
        }

    /* ensembles at given times, realizations on threads */
    const int64_t times[] = {1, 3, 7};
    int64_t out[4 * 3 * 2];
    CHECK(or_ensemble_at(32, 32, 0.9, 0.1, 5, 4, times, 3, 0, out) == 0);
    CHECK(or_ensemble_at(32, 32, 0.9, 0.1, 5, 4, times, 3, 1, out) == 0);
    CHECK(or_ensemble_at(32, 32, 0.9, 0.1, 5, 4, times, 3, 2, out) == 0);
    const int64_t bad_times[] = {3, 3};
    CHECK(or_ensemble_at(32, 32, 0.9, 0.1, 5, 4, bad_times, 2, 0, out) == -2);

    /* a wrapping window against the whole lattice */
    /* each sweep loses less than two blocks per axis: 5 blocks leave one after two */
    const int64_t Lx = 2048, Ly = 1536, Wx = 1536, Wy = 1280, wx0 = 1700, wy0 = -100;
    uint8_t *full = malloc((size_t)(Lx * Ly)), *win = malloc((size_t)(Wx * Wy));
    or_flat(full, Lx, Ly);
    for (int64_t v = 0; v < Wy; ++v)
        for (int64_t u = 0; u < Wx; ++u)
            win[v * Wx + u] = full[(((wy0 + v) % Ly + Ly) % Ly) * Lx + ((wx0 + u) % Lx + Lx) % Lx];
    int64_t vx0 = 0, vy0 = 0, vx1 = Wx, vy1 = Wy, Hw = 0, Hf = 0;
    const uint64_t Tp = or_threshold(0.8), Tq = or_threshold(0.3);
    for (uint32_t s = 0; s < 2; ++s) {
        CHECK(or_sweep(full, Lx, Ly, Tp, Tq, 3, s, &Hf, NULL, NULL, 0, 1) == 0);
        CHECK(or_window_sweep(win, Wx, Wy, wx0, wy0, Lx, Ly, Tp, Tq, 3, s, &vx0, &vy0, &vx1,
                              &vy1, &Hw, 1) == 0);
    }
    CHECK(vx1 > vx0 && vy1 > vy0);
    for (int64_t v = vy0; v < vy1; ++v)
        for (int64_t u = vx0; u < vx1; ++u)
            CHECK(win[v * Wx + u] ==
                  full[(((wy0 + v) % Ly + Ly) % Ly) * Lx + ((wx0 + u) % Lx + Lx) % Lx]);
    CHECK(or_window_sweep(win, Wx + Lx, Wy, wx0, wy0, Lx, Ly, Tp, Tq, 3, 2, &vx0, &vy0, &vx1,
                          &vy1, &Hw, 0) == -2);
    free(full);
    free(win);

    if (fails) return 1;
    printf("oracle ok\n");
    return 0;
}
