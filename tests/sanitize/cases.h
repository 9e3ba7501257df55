/* Synthetic networks for the sanitizer drivers (CPU only): a random tree
 * plus extra branches, generators, loads, storage units and devices, from
 * a fixed linear congruential generator.  Shapes only: the drivers look for
 * memory and undefined-behaviour errors, not values. */
#pragma once
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int32_t N, L, G, S, D;
    double *pd, *qd, *gs, *bs, *vmin, *vmax;
    int32_t ref_bus[1];
    int32_t *f_bus, *t_bus, *gen_bus, *stor_bus, *dev_bus;
    double *r, *x, *b, *tap, *shift, *rate, *angmin, *angmax;
    double *pmin, *pmax, *qmin, *qmax, *c2, *c1, *c0;
    double *st[13]; /* emax chmax dismax rating qmin qmax eta_c eta_d r x ploss qloss e0 */
    double *dv[8];  /* cp cq cost lo hi ramp init_lo init_hi */
} san_net;

static uint64_t san_state;
static double san_u(void) {
    san_state = san_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(san_state >> 11) * (1.0 / 9007199254740992.0);
}
static double *san_vec(int n, double lo, double hi) {
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; i++) v[i] = lo + (hi - lo) * san_u();
    return v;
}

/* hub != 0: bus 0 also joins `hub` extra branches (a segment wider than a
 * wave); parallel branches are allowed. */
static void san_make(san_net *n, int N, int extra, int G, int S, int D, int hub, uint64_t seed) {
    san_state = seed;
    n->N = N; n->L = N - 1 + extra + hub; n->G = G; n->S = S; n->D = D;
    int L = n->L;
    n->f_bus = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    n->t_bus = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    int l = 0;
    for (int i = 1; i < N; i++, l++) { n->f_bus[l] = (int32_t)(san_u() * i); n->t_bus[l] = i; }
    for (int k = 0; k < extra; k++, l++) {
        int a = (int)(san_u() * N), c = (int)(san_u() * N);
        if (a == c) c = (a + 1) % N;
        n->f_bus[l] = a; n->t_bus[l] = c;
    }
    for (int k = 0; k < hub; k++, l++) { n->f_bus[l] = 0; n->t_bus[l] = 1 + k % (N - 1); }
    n->pd = san_vec(N, 0, 0.5); n->qd = san_vec(N, 0, 0.15); n->gs = san_vec(N, -0.05, 0.05);
    n->bs = san_vec(N, -0.05, 0.05); n->vmin = san_vec(N, 0.9, 0.9); n->vmax = san_vec(N, 1.1, 1.1);
    n->r = san_vec(L, 0.005, 0.05); n->x = san_vec(L, 0.02, 0.3); n->b = san_vec(L, 0, 0.05);
    n->tap = san_vec(L, 0.9, 1.1); n->shift = san_vec(L, -0.1, 0.1); n->rate = san_vec(L, 0.5, 2);
    n->angmin = san_vec(L, -0.5, -0.5); n->angmax = san_vec(L, 0.5, 0.5);
    n->gen_bus = (int32_t *)malloc(sizeof(int32_t) * (size_t)(G > 0 ? G : 1));
    for (int k = 0; k < G; k++) n->gen_bus[k] = (int32_t)(san_u() * N);
    n->ref_bus[0] = G > 0 ? n->gen_bus[0] : 0;
    n->pmin = san_vec(G, 0, 0); n->pmax = san_vec(G, 3, 3); n->qmin = san_vec(G, -1, -1);
    n->qmax = san_vec(G, 1, 1); n->c2 = san_vec(G, 0.01, 0.1); n->c1 = san_vec(G, 10, 40); n->c0 = san_vec(G, 0, 1);
    n->stor_bus = (int32_t *)malloc(sizeof(int32_t) * (size_t)(S > 0 ? S : 1));
    for (int k = 0; k < S; k++) n->stor_bus[k] = k == 0 ? 0 : (int32_t)(san_u() * N);
    static const double lo[13] = {0.5, 0.2, 0.2, 0.3, -0.1, 0.1, 0.9, 0.9, 0, 0, 0, 0, 0.2};
    static const double hi[13] = {1.0, 0.4, 0.4, 0.5, -0.1, 0.1, 0.95, 0.95, 0.02, 0.05, 1e-3, 1e-3, 0.3};
    for (int k = 0; k < 13; k++) n->st[k] = san_vec(S, lo[k], hi[k]);
    n->dev_bus = (int32_t *)malloc(sizeof(int32_t) * (size_t)(D > 0 ? D : 1));
    for (int k = 0; k < D; k++) n->dev_bus[k] = k == 0 ? 0 : (int32_t)(san_u() * N);
    static const double dlo[8] = {1, 0, -50, 0, 0.5, 0.1, 0, 0}, dhi[8] = {1, 0.3, -10, 0, 0.5, 0.1, 0, 0};
    for (int k = 0; k < 8; k++) n->dv[k] = san_vec(D, dlo[k], dhi[k]);
}

static void san_free(san_net *n) {
    void *p[] = {n->pd, n->qd, n->gs, n->bs, n->vmin, n->vmax, n->f_bus, n->t_bus, n->gen_bus, n->stor_bus,
                 n->dev_bus, n->r, n->x, n->b, n->tap, n->shift, n->rate, n->angmin, n->angmax, n->pmin, n->pmax,
                 n->qmin, n->qmax, n->c2, n->c1, n->c0};
    for (size_t k = 0; k < sizeof p / sizeof p[0]; k++) free(p[k]);
    for (int k = 0; k < 13; k++) free(n->st[k]);
    for (int k = 0; k < 8; k++) free(n->dv[k]);
}
