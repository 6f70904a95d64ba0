/* Plain C99 use of include/sv.h: host-only entry points (no GPU needed).
 * Prints "ok" when the gate table and the paper-rule fusion behave. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "sv.h"

int main(void)
{
    sv_gate g[10];
    int i = 0;
    memset(g, 0, sizeof g);
    /* the paper's compress example: CPHASE(1) on all pairs of 5 qubits */
    for (int a = 0; a < 5; ++a)
        for (int b = a + 1; b < 5; ++b) {
            g[i].kind = SV_G_CPHASE;
            g[i].k = 2;
            g[i].q[0] = a;
            g[i].q[1] = b;
            g[i].params[0] = 1.0;
            g[i].param = -1;
            ++i;
        }
    sv_plan *p = NULL;
    if (sv_fuse(g, 10, 5, 3, SV_RULE_PAPER, &p) != SV_OK) {
        printf("fuse failed: %s\n", sv_last_error());
        return 1;
    }
    int nb = 0;
    sv_plan_num_blocks(p, &nb);
    const int want[4][3] = {{0, 1, 2}, {0, 3, 4}, {1, 3, 4}, {2, 3, 4}};
    if (nb != 4) return 2;
    for (int b = 0; b < nb; ++b) {
        int32_t k, q[SV_MAX_K], nm;
        sv_plan_block(p, b, &k, q, &nm);
        if (k != 3 || q[0] != want[b][0] || q[1] != want[b][1] || q[2] != want[b][2]) return 3;
    }
    sv_plan_free(p);
    /* H matrix */
    sv_gate h;
    memset(&h, 0, sizeof h);
    h.kind = SV_G_H;
    h.k = 1;
    h.param = -1;
    double m[8];
    if (sv_gate_matrix(&h, m) != SV_OK) return 4;
    if (fabs(m[0] - sqrt(0.5)) > 1e-15 || fabs(m[6] + sqrt(0.5)) > 1e-15) return 5;
    /* invalid: repeated qubit */
    g[0].q[1] = 0;
    if (sv_fuse(g, 1, 5, 3, SV_RULE_PAPER, &p) != SV_ERR_QUBIT) return 6;
    printf("ok %d\n", sv_version());
    return 0;
}
