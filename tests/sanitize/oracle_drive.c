/* Exercises the FP64 oracle under AddressSanitizer / UBSan (built and run by
 * tests/test_oracle_sanitized.py): plain Shan-Chen with source and merges, the barrier, gravity,
 * two components, film geometry and labelling, in 2D and 3D. */
#include <stdio.h>
#include <stdlib.h>
#include "sc_oracle.h"

static void run(int q, int nx, int ny, int nz, int mode)
{
    orc_sim* s = orc_create(q, nx, ny, nz, 1.0, mode == 3 ? 0.0 : -5.0, mode == 3 ? 1.0 : 1.93,
                            mode == 3 ? 0.05 : 0.16, 1e-3, 7, 0.0, 10, 8);
    if (!s) { printf("create failed\n"); exit(1); }
    if (mode == 1) orc_set_barrier(s, 1, 3);
    if (mode == 2) { double g[3] = {0.0, -1e-5, 0.0}; orc_set_gravity(s, g, 0.0); }
    if (mode == 3) orc_set_two_component(s, 1.5, 0.8, 1.0, 0.05);
    double c[6] = {nx / 2.0 - 8.5, ny / 2.0 - 0.5, q == 19 ? nz / 2.0 - 0.5 : 0.0,
                   nx / 2.0 + 7.5, ny / 2.0 - 0.5, q == 19 ? nz / 2.0 - 0.5 : 0.0};
    double r[2] = {5.0, 5.0}, b[2] = {1.0, 1.0};
    orc_seed_nuclei(s, 2, c, r, b, 1e-3);
    orc_step(s, 60);
    int64_t N = orc_num_nodes(s);
    double* rho = malloc(sizeof(double) * N);
    double* u = malloc(sizeof(double) * N * 3);
    double* p = malloc(sizeof(double) * N);
    double* lap = malloc(sizeof(double) * N);
    double tot[4];
    orc_fields(s, rho, u, tot);
    orc_laplacian_p(s, p, lap);
    orc_bubbles(s, NULL, 0);
    orc_event ev[4];
    int ne = orc_events(s, ev, 4);
    double h = 0, rd = 0;
    int nl = 0;
    int fg = orc_film_geometry(s, 0, 1, &h, &rd, &nl);
    printf("q %d mode %d: M %.6f events %d film rc %d h %.3f\n", q, mode, tot[0], ne, fg, h);
    free(rho); free(u); free(p); free(lap);
    orc_destroy(s);
}

int main(void)
{
    for (int mode = 0; mode < 4; ++mode) {
        run(9, 48, 32, 1, mode);
        run(19, 40, 20, 18, mode);
    }
    uint8_t mask[6 * 5 * 4];
    uint32_t lab[6 * 5 * 4];
    for (int i = 0; i < 120; ++i) mask[i] = (uint8_t)((i * 37 + 11) % 7 < 3);
    printf("labels %lld %lld\n", (long long)orc_label_mask(9, 6, 20, 1, mask, lab),
           (long long)orc_label_mask(19, 6, 5, 4, mask, lab));
    return 0;
}
