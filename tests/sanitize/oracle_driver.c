/* Sanitizer driver for the CPU oracle: built with gcc and
 * -fsanitize=address,undefined by tests/test_sanitize.py, evaluating every
 * callback of static, multi-period, contingency, rectangular, storage and
 * device models, with bounds, plus malformed inputs. */
#include <stdio.h>

#include "../../oracle/opf_oracle.c"
#include "cases.h"

static int run(const san_net *n, or_case cs, int expect_ok) {
    cs.n_bus = n->N; cs.n_branch = n->L; cs.n_gen = n->G; cs.n_ref = 1;
    cs.pd = n->pd; cs.qd = n->qd; cs.gs = n->gs; cs.bs = n->bs; cs.vmin = n->vmin; cs.vmax = n->vmax;
    cs.ref_bus = n->ref_bus; cs.f_bus = n->f_bus; cs.t_bus = n->t_bus;
    cs.r = n->r; cs.x = n->x; cs.b = n->b; cs.tap = n->tap; cs.shift = n->shift; cs.rate_a = n->rate;
    cs.angmin = n->angmin; cs.angmax = n->angmax; cs.gen_bus = n->gen_bus;
    cs.pmin = n->pmin; cs.pmax = n->pmax; cs.qmin = n->qmin; cs.qmax = n->qmax;
    cs.c2 = n->c2; cs.c1 = n->c1; cs.c0 = n->c0;
    int64_t nv, m;
    if (or_dims(&cs, &nv, &m)) return expect_ok ? 1 : 0;
    double *x = san_vec((int)nv, 0.5, 1.0), *y = san_vec((int)m, -1, 1);
    double *lv = san_vec((int)nv, 0, 0), *uv = san_vec((int)nv, 0, 0), *x0 = san_vec((int)nv, 0, 0);
    double *lc = san_vec((int)m, 0, 0), *uc = san_vec((int)m, 0, 0);
    int rc = or_bounds(&cs, lv, uv, lc, uc, x0);
    or_result *res = rc ? NULL : or_eval(&cs, x, y, 0.7, W_OBJ | W_CONS | W_JAC | W_HESS);
    int ok = res != NULL;
    or_free(res);
    free(x); free(y); free(lv); free(uv); free(x0); free(lc); free(uc);
    if (ok != expect_ok) {
        fprintf(stderr, "unexpected status: %s\n", or_error());
        return 1;
    }
    return 0;
}

int main(void) {
    int bad = 0;
    san_net a, b;
    san_make(&a, 40, 15, 8, 0, 0, 0, 1);
    san_make(&b, 90, 20, 15, 5, 4, 70, 2);
    double pdt[3 * 90], qdt[3 * 90];
    for (int k = 0; k < 270; k++) { pdt[k] = b.pd[k % 90]; qdt[k] = b.qd[k % 90]; }
    int32_t out[2] = {3, 7};
    or_case base;
    memset(&base, 0, sizeof base);
    base.n_periods = 1;
    or_case mp = base; mp.n_periods = 3; mp.pd_t = pdt; mp.qd_t = qdt; mp.ramp_ratio = 0.2;
    or_case sc = base; sc.n_cont = 2; sc.outaged = out;
    or_case rect = mp; rect.form = 1;
    or_case ext = mp;
    ext.n_stor = b.S; ext.stor_bus = b.stor_bus;
    ext.stor_emax = b.st[0]; ext.stor_chmax = b.st[1]; ext.stor_dismax = b.st[2]; ext.stor_rating = b.st[3];
    ext.stor_qmin = b.st[4]; ext.stor_qmax = b.st[5]; ext.stor_eta_c = b.st[6]; ext.stor_eta_d = b.st[7];
    ext.stor_r = b.st[8]; ext.stor_x = b.st[9]; ext.stor_ploss = b.st[10]; ext.stor_qloss = b.st[11];
    ext.stor_e0 = b.st[12]; ext.stor_dt = 0.5; ext.stor_comp = 1;
    ext.n_dev = b.D; ext.dev_bus = b.dev_bus; ext.dev_cp = b.dv[0]; ext.dev_cq = b.dv[1]; ext.dev_cost = b.dv[2];
    ext.dev_lo = b.dv[3]; ext.dev_hi = b.dv[4]; ext.dev_ramp = b.dv[5]; ext.dev_init_lo = b.dv[6];
    ext.dev_init_hi = b.dv[7];
    bad |= run(&a, base, 1);
    bad |= run(&a, sc, 1);
    bad |= run(&b, mp, 1);
    bad |= run(&b, rect, 1);
    bad |= run(&b, ext, 1);
    or_case bad1 = ext; bad1.form = 1;
    bad |= run(&b, bad1, 0);
    b.f_bus[4] = 500;
    bad |= run(&b, mp, 0);
    san_free(&a);
    san_free(&b);
    printf(bad ? "oracle driver: FAILED\n" : "oracle driver: ok\n");
    return bad;
}
