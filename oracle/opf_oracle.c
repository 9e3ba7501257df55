/*
 * CPU ORACLE for the AC-OPF NLP callbacks, polar and rectangular forms.
 * TEST INFRASTRUCTURE ONLY:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library; the product path never does.
 *
 * What it computes (the callbacks of the NLPModels template, Listing 1):
 *   f(x)          objective, sum of generator costs c2 pg^2 + c1 pg + c0
 *                 (Listing 3, the objective line)
 *   grad f(x)     dense gradient
 *   c(x)          every constraint row, in the order Listing 3 creates them:
 *                 reference angle, four branch-flow definitions, angle
 *                 difference, active and reactive balance (demand term, then
 *                 the arc terms and the generator terms that constraint!
 *                 adds), from- and to-side thermal limits; multi-period
 *                 models repeat every block per period (entity fastest, the
 *                 balance-row index bus + Nbus*(t-1) of the user-extension
 *                 example in Sec. III-D) and append generator ramp rows
 *                 pg_t - pg_{t-1} (the mpopf ramp limit, Sec. III-C2);
 *                 contingency copies repeat every block except pg.
 *                 The rectangular form (form = :rect, Sec. III-C1) takes
 *                 bus variables (vr, vi) for (va, vm) and rows of
 *                 PowerModels' ACR formulation (see row_value_rect).
 *                 Storage units (Sec. III-C3, the storage model of Geth,
 *                 Coffrin and Fobes 2020 that the paper cites) and linear
 *                 user-extension devices (Sec. III-D, Listing 10) add
 *                 their variable and row blocks after the others and their
 *                 terms to the balance rows (see row_value_ext).
 *   J(x)          sparse Jacobian values, sorted by (row, col)
 *   H(x, y, s)    lower triangle of s * hess f + sum_i y_i hess c_i, sorted by
 *                 (row, col), duplicates merged (hess! with obj_weight,
 *                 Listing 1)
 *
 * How: every row is written out once as a function of its own variables,
 * evaluated in hyper-dual arithmetic (Fike and Alonso, AIAA 2011): seeding
 * e1 and e2 gives exact first and second partial derivatives with no
 * truncation error.  The Jacobian support of a row is the list of variables
 * it reads; its Hessian support is the list of variable pairs that appear
 * together inside a nonlinear term (all pairs of the four voltage variables
 * of a flow row, the squared voltage of a balance row, the two squares of a
 * thermal row, the squared pg of a cost term).  Entries are structural: they
 * stay in the pattern when their value happens to be zero.
 *
 * Each hyper-dual also carries a magnitude companion: the same arithmetic
 * applied to absolute values, i.e. the sum of |terms| that produced each
 * component.  It is returned as the per-output scale S used by the
 * scale-aware tolerance |v - v*| <= rtol * max(|v*|, S) + atol.
 *
 * Branch physics: the textbook pi model with an ideal transformer on the
 * from side, line charging split b/2 per side and no series-shunt
 * conductance, as in the PowerModels formulation the paper follows.
 *
 * Plain C99, compiled with -O2 -ffp-contract=off (no FMA contraction).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* input                                                               */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t n_bus, n_branch, n_gen, n_ref;
    const double *pd, *qd, *gs, *bs, *vmin, *vmax;
    const int32_t *ref_bus;
    const int32_t *f_bus, *t_bus;
    const double *r, *x, *b, *tap, *shift, *rate_a, *angmin, *angmax;
    const int32_t *gen_bus;
    const double *pmin, *pmax, *qmin, *qmax, *c2, *c1, *c0;
    int32_t n_periods;          /* >= 1 */
    const double *pd_t, *qd_t;  /* [n_periods * n_bus] bus fastest, or NULL */
    double ramp_ratio;
    int32_t n_cont;             /* contingency copies (0 = none) */
    const int32_t *outaged;     /* [n_cont] */
    int32_t form;               /* 0 = polar (va, vm), 1 = rectangular (vr, vi) */
    /* storage units (polar form, no contingency copies) */
    int32_t n_stor;
    const int32_t *stor_bus;
    const double *stor_emax, *stor_chmax, *stor_dismax, *stor_rating, *stor_qmin, *stor_qmax;
    const double *stor_eta_c, *stor_eta_d, *stor_r, *stor_x, *stor_ploss, *stor_qloss, *stor_e0;
    double stor_dt;             /* duration of a period */
    int32_t stor_comp;          /* 1: add the complementarity rows sc * sd */
    /* linear user-extension devices (no contingency copies) */
    int32_t n_dev;
    const int32_t *dev_bus;     /* every device enters both balance rows of its bus */
    const double *dev_cp, *dev_cq, *dev_cost, *dev_lo, *dev_hi, *dev_ramp, *dev_init_lo, *dev_init_hi;
} or_case;

typedef struct {
    int64_t n, m, nnzj, nnzh;
    double f, fscale;
    double *g;                 /* [n] */
    double *c, *cscale;        /* [m] */
    int32_t *jrow, *jcol;
    double *jval, *jscale;     /* [nnzj] */
    int32_t *hrow, *hcol;
    double *hval, *hscale;     /* [nnzh] */
} or_result;

static char g_err[256];
const char *or_error(void) { return g_err; }
static int fail(const char *msg) {
    snprintf(g_err, sizeof g_err, "%s", msg);
    return -1;
}

/* ------------------------------------------------------------------ */
/* hyper-dual numbers with magnitude companion                        */
/*   value = a + b e1 + c e2 + d e1 e2,  e1^2 = e2^2 = 0               */
/* ------------------------------------------------------------------ */
typedef struct {
    double a, b, c, d;      /* value parts */
    double ma, mb, mc, md;  /* magnitudes (sums of |terms|) */
} hd;

static hd hd_cst(double v) {
    hd z = {v, 0, 0, 0, fabs(v), 0, 0, 0};
    return z;
}
static hd hd_var(double v, double s1, double s2) {
    hd z = {v, s1, s2, 0, fabs(v), fabs(s1), fabs(s2), 0};
    return z;
}
static hd hd_add(hd x, hd y) {
    hd z = {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d,
            x.ma + y.ma, x.mb + y.mb, x.mc + y.mc, x.md + y.md};
    return z;
}
static hd hd_sub(hd x, hd y) {
    hd z = {x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d,
            x.ma + y.ma, x.mb + y.mb, x.mc + y.mc, x.md + y.md};
    return z;
}
static hd hd_mul(hd x, hd y) {
    hd z;
    z.a = x.a * y.a;
    z.b = x.a * y.b + x.b * y.a;
    z.c = x.a * y.c + x.c * y.a;
    z.d = x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a;
    z.ma = x.ma * y.ma;
    z.mb = x.ma * y.mb + x.mb * y.ma;
    z.mc = x.ma * y.mc + x.mc * y.ma;
    z.md = x.ma * y.md + x.mb * y.mc + x.mc * y.mb + x.md * y.ma;
    return z;
}
/* 1 / x: value 1/a, first parts -b/a^2, -c/a^2, second part
 * 2 b c / a^3 - d / a^2 (the Taylor expansion of 1/(a + h) to second order
 * in the two directions).  Magnitudes: the same expressions on |parts|. */
static hd hd_inv(hd x) {
    hd r;
    double a = x.a, a2 = a * a, a3 = a2 * a, aa = fabs(a);
    r.a = 1.0 / a;
    r.b = -x.b / a2;
    r.c = -x.c / a2;
    r.d = 2.0 * x.b * x.c / a3 - x.d / a2;
    r.ma = 1.0 / aa;
    r.mb = x.mb / a2;
    r.mc = x.mc / a2;
    r.md = 2.0 * x.mb * x.mc / (a2 * aa) + x.md / a2;
    return r;
}
static hd hd_scale(double s, hd x) {
    double as = fabs(s);
    hd z = {s * x.a, s * x.b, s * x.c, s * x.d,
            as * x.ma, as * x.mb, as * x.mc, as * x.md};
    return z;
}
/* g(x) for g = sin or cos: g(a) + g'(a)(b e1 + c e2) + (g'(a) d + g''(a) b c) e1 e2.
 * Magnitudes: sin and cos are single terms of the rows they enter, so each
 * part's companion is the absolute value of the term itself, |g(a)|,
 * |g'(a)| |b|, ... carried through the chain rule term by term (the literal
 * sum of |contributions|; the argument's own magnitude plays no part). */
static hd hd_trig(hd x, double g0, double g1, double g2) {
    hd z;
    z.a = g0;
    z.b = g1 * x.b;
    z.c = g1 * x.c;
    z.d = g1 * x.d + g2 * x.b * x.c;
    z.ma = fabs(g0);
    z.mb = fabs(g1) * x.mb;
    z.mc = fabs(g1) * x.mc;
    z.md = fabs(g1) * x.md + fabs(g2) * x.mb * x.mc;
    return z;
}
static hd hd_sin(hd x) { return hd_trig(x, sin(x.a), cos(x.a), -sin(x.a)); }
static hd hd_cos(hd x) { return hd_trig(x, cos(x.a), -sin(x.a), -cos(x.a)); }

/* ------------------------------------------------------------------ */
/* layout: variable and constraint blocks                              */
/* ------------------------------------------------------------------ */
/* R_ANGL (the lower angle-difference row) and R_VMAG (voltage magnitude)
 * exist in the rectangular form only; in the polar form they are empty. */
/* Storage rows (per unit and period): R_SOC state of charge, R_SLP / R_SLQ
 * active and reactive loss rows, R_STH thermal limit, R_SCMP the optional
 * complementarity row; device rows: R_DRAMP ramp (periods 1..T-1), R_DINIT
 * initial value (period 0). */
enum { R_REF, R_PFR, R_QFR, R_PTO, R_QTO, R_ANG, R_ANGL, R_BALP, R_BALQ, R_THF, R_THT, R_VMAG, R_RAMP,
       R_SOC, R_SLP, R_SLQ, R_STH, R_SCMP, R_DRAMP, R_DINIT, R_NBLK };

typedef struct {
    int N, L, G, R, T, K, nrep, npg, rect, S, D;
    int64_t xva, xvm, xpg, xqg, xp, xq, n;
    /* storage blocks ps, qs, qsc, se, sc, sd and the device block u, each
     * S * nrep (D * nrep), unit fastest */
    int64_t xps, xqs, xqsc, xse, xsc, xsd, xu;
    int64_t cblk[R_NBLK + 1]; /* start row of every constraint block; cblk[R_NBLK] = m */
} layout;

static int make_layout(const or_case *cs, layout *ly) {
    if (cs->n_bus < 1 || cs->n_branch < 0 || cs->n_gen < 0 || cs->n_ref < 0)
        return fail("negative sizes");
    if (cs->n_periods < 1) return fail("n_periods must be >= 1");
    if (cs->n_cont < 0) return fail("n_cont must be >= 0");
    if (cs->n_periods > 1 && cs->n_cont > 0)
        return fail("periods and contingency copies are not combined");
    if (cs->form != 0 && cs->form != 1) return fail("form must be 0 (polar) or 1 (rectangular)");
    if (cs->n_stor < 0 || cs->n_dev < 0) return fail("negative storage or device count");
    if ((cs->n_stor > 0 || cs->n_dev > 0) && cs->n_cont > 0)
        return fail("storage and devices are not combined with contingency copies");
    if (cs->n_stor > 0 && cs->form != 0) return fail("storage units take the polar form");
    ly->rect = cs->form;
    ly->S = cs->n_stor;
    ly->D = cs->n_dev;
    ly->N = cs->n_bus; ly->L = cs->n_branch; ly->G = cs->n_gen; ly->R = cs->n_ref;
    ly->T = cs->n_periods; ly->K = cs->n_cont;
    ly->nrep = cs->n_periods > 1 ? cs->n_periods : cs->n_cont + 1;
    ly->npg = cs->n_cont > 0 ? 1 : ly->nrep;
    int64_t N = ly->N, L = ly->L, G = ly->G, R = ly->R, nr = ly->nrep;
    ly->xva = 0;
    ly->xvm = N * nr;
    ly->xpg = 2 * N * nr;
    ly->xqg = ly->xpg + G * ly->npg;
    ly->xp = ly->xqg + G * nr;
    ly->xq = ly->xp + 2 * L * nr;
    int64_t S = ly->S, D = ly->D;
    ly->xps = ly->xq + 2 * L * nr;
    ly->xqs = ly->xps + S * nr;
    ly->xqsc = ly->xqs + S * nr;
    ly->xse = ly->xqsc + S * nr;
    ly->xsc = ly->xse + S * nr;
    ly->xsd = ly->xsc + S * nr;
    ly->xu = ly->xsd + S * nr;
    ly->n = ly->xu + D * nr;
    int64_t rc = ly->rect, T1 = ly->T - 1;
    int64_t sizes[R_NBLK] = {R * nr, L * nr, L * nr, L * nr, L * nr, L * nr, rc * L * nr,
                             N * nr, N * nr, L * nr, L * nr, rc * N * nr,
                             G * T1, S * nr, S * nr, S * nr, S * nr, (cs->stor_comp ? S : 0) * nr,
                             D * T1, D};
    ly->cblk[0] = 0;
    for (int k = 0; k < R_NBLK; k++) ly->cblk[k + 1] = ly->cblk[k] + sizes[k];
    return 0;
}
/* The two bus blocks: (va, vm) in the polar form, (vr, vi) in the
 * rectangular form (same positions). */
static int64_t col_va(const layout *l, int i, int r) { return l->xva + i + (int64_t)l->N * r; }
static int64_t col_vm(const layout *l, int i, int r) { return l->xvm + i + (int64_t)l->N * r; }
static int64_t col_vr(const layout *l, int i, int r) { return col_va(l, i, r); }
static int64_t col_vi(const layout *l, int i, int r) { return col_vm(l, i, r); }
static int64_t col_pg(const layout *l, int k, int r) {
    return l->xpg + k + (int64_t)l->G * (l->npg == 1 ? 0 : r);
}
static int64_t col_qg(const layout *l, int k, int r) { return l->xqg + k + (int64_t)l->G * r; }
static int64_t col_p(const layout *l, int a, int r) { return l->xp + a + 2 * (int64_t)l->L * r; }
static int64_t col_q(const layout *l, int a, int r) { return l->xq + a + 2 * (int64_t)l->L * r; }
/* storage unit u and device d in period r */
static int64_t col_ps(const layout *l, int u, int r) { return l->xps + u + (int64_t)l->S * r; }
static int64_t col_qs(const layout *l, int u, int r) { return l->xqs + u + (int64_t)l->S * r; }
static int64_t col_qsc(const layout *l, int u, int r) { return l->xqsc + u + (int64_t)l->S * r; }
static int64_t col_se(const layout *l, int u, int r) { return l->xse + u + (int64_t)l->S * r; }
static int64_t col_sc(const layout *l, int u, int r) { return l->xsc + u + (int64_t)l->S * r; }
static int64_t col_sd(const layout *l, int u, int r) { return l->xsd + u + (int64_t)l->S * r; }
static int64_t col_u(const layout *l, int d, int r) { return l->xu + d + (int64_t)l->D * r; }

/* ------------------------------------------------------------------ */
/* branch admittance terms of the pi model                             */
/* ------------------------------------------------------------------ */
typedef struct { double Gff, Bff, Gft, Bft, Gtt, Btt, Gtf, Btf; } bcoef;

static bcoef branch_coef(const or_case *cs, int l, int rep) {
    bcoef k;
    /* a contingency copy s >= 1 takes its outaged branch out of service */
    if (cs->n_cont > 0 && rep >= 1 && cs->outaged[rep - 1] == l) {
        memset(&k, 0, sizeof k);
        return k;
    }
    double r = cs->r[l], x = cs->x[l];
    double z = r * r + x * x;
    double g = r / z, b = -x / z;            /* series admittance g + jb */
    double tr = cs->tap[l] * cos(cs->shift[l]);
    double ti = cs->tap[l] * sin(cs->shift[l]);
    double tm = cs->tap[l] * cs->tap[l];     /* |tap|^2 */
    double bfr = cs->b[l] / 2, bto = cs->b[l] / 2, gfr = 0.0, gto = 0.0;
    k.Gff = (g + gfr) / tm;
    k.Bff = (b + bfr) / tm;
    k.Gft = (-g * tr + b * ti) / tm;
    k.Bft = (-b * tr - g * ti) / tm;
    k.Gtt = g + gto;
    k.Btt = b + bto;
    k.Gtf = (-g * tr - b * ti) / tm;
    k.Btf = (-b * tr + g * ti) / tm;
    return k;
}

/* ------------------------------------------------------------------ */
/* rows                                                                */
/* ------------------------------------------------------------------ */
typedef struct {
    int blk, ent, rep;   /* block, entity (ref index / branch / bus / gen), replica */
    int nsup;
    int narc;            /* balance rows: number of arc terms */
    int nbv;             /* balance rows: leading bus variables (1 polar: vm; 2 rect: vr, vi) */
    int ngen, nstor;     /* balance rows: generator and storage terms */
    const int32_t *devs; /* balance rows: the devices of the device terms (the rest of the row) */
    int64_t sup[64 + 16]; /* variable columns, in term order (filled by row_support) */
    int64_t *big;         /* used instead of sup when a balance row is long */
} row_t;

typedef struct {
    /* arcs, generators, storage units and devices at each bus, for the
     * balance rows */
    int32_t *arc_ptr, *arc_idx, *gen_ptr, *gen_idx, *st_ptr, *st_idx, *dv_ptr, *dv_idx;
} adjacency;

/* Entities e with bus(e) listed per bus in increasing index: ptr [N+1],
 * idx [count]. */
static int bus_lists(int N, int count, const int32_t *bus, int32_t **ptr, int32_t **idx) {
    *ptr = calloc((size_t)N + 1, sizeof(int32_t));
    *idx = malloc(sizeof(int32_t) * (size_t)(count + 1));
    if (!*ptr || !*idx) return fail("out of memory");
    for (int e = 0; e < count; e++) (*ptr)[bus[e] + 1]++;
    for (int i = 0; i < N; i++) (*ptr)[i + 1] += (*ptr)[i];
    int32_t *fill = calloc((size_t)N + 1, sizeof(int32_t));
    if (!fill) return fail("out of memory");
    for (int e = 0; e < count; e++) (*idx)[(*ptr)[bus[e]] + fill[bus[e]]++] = e;
    free(fill);
    return 0;
}

static int build_adjacency(const or_case *cs, adjacency *adj) {
    int N = cs->n_bus, L = cs->n_branch, G = cs->n_gen;
    adj->arc_ptr = calloc((size_t)N + 1, sizeof(int32_t));
    adj->arc_idx = malloc(sizeof(int32_t) * (size_t)(2 * L + 1));
    adj->gen_ptr = calloc((size_t)N + 1, sizeof(int32_t));
    adj->gen_idx = malloc(sizeof(int32_t) * (size_t)(G + 1));
    if (!adj->arc_ptr || !adj->arc_idx || !adj->gen_ptr || !adj->gen_idx) return fail("out of memory");
    /* arc a < L sits at f_bus[a]; arc L + l sits at t_bus[l].  Lists are in
     * increasing arc (generator) index, the order constraint! adds them. */
    for (int a = 0; a < 2 * L; a++) {
        int bus = a < L ? cs->f_bus[a] : cs->t_bus[a - L];
        adj->arc_ptr[bus + 1]++;
    }
    for (int i = 0; i < N; i++) adj->arc_ptr[i + 1] += adj->arc_ptr[i];
    int32_t *fill = calloc((size_t)N, sizeof(int32_t));
    for (int a = 0; a < 2 * L; a++) {
        int bus = a < L ? cs->f_bus[a] : cs->t_bus[a - L];
        adj->arc_idx[adj->arc_ptr[bus] + fill[bus]++] = a;
    }
    memset(fill, 0, sizeof(int32_t) * (size_t)N);
    for (int k = 0; k < G; k++) adj->gen_ptr[cs->gen_bus[k] + 1]++;
    for (int i = 0; i < N; i++) adj->gen_ptr[i + 1] += adj->gen_ptr[i];
    for (int k = 0; k < G; k++) {
        int bus = cs->gen_bus[k];
        adj->gen_idx[adj->gen_ptr[bus] + fill[bus]++] = k;
    }
    free(fill);
    if (bus_lists(N, cs->n_stor, cs->stor_bus, &adj->st_ptr, &adj->st_idx)) return -1;
    if (bus_lists(N, cs->n_dev, cs->dev_bus, &adj->dv_ptr, &adj->dv_idx)) return -1;
    return 0;
}
static void free_adjacency(adjacency *adj) {
    free(adj->arc_ptr); free(adj->arc_idx); free(adj->gen_ptr); free(adj->gen_idx);
    free(adj->st_ptr); free(adj->st_idx); free(adj->dv_ptr); free(adj->dv_idx);
}

static int64_t *row_sup(row_t *rw) { return rw->big ? rw->big : rw->sup; }

/* Fill the variable list of a row (term order). */
static int row_support(const or_case *cs, const layout *ly, const adjacency *adj, row_t *rw) {
    int e = rw->ent, r = rw->rep, L = ly->L;
    int64_t *s = rw->sup;
    rw->big = NULL;
    rw->narc = 0;
    rw->nbv = ly->rect ? 2 : 1;
    switch (rw->blk) {
    case R_REF:
        /* polar: va_r; rectangular: vi_r (a zero angle with vr > 0) */
        rw->nsup = 1;
        s[0] = ly->rect ? col_vi(ly, cs->ref_bus[e], r) : col_va(ly, cs->ref_bus[e], r);
        break;
    case R_PFR: case R_QFR: case R_PTO: case R_QTO: {
        int arc = (rw->blk == R_PFR || rw->blk == R_QFR) ? e : L + e;
        int isp = (rw->blk == R_PFR || rw->blk == R_PTO);
        rw->nsup = 5;
        s[0] = isp ? col_p(ly, arc, r) : col_q(ly, arc, r);
        if (ly->rect) { /* (vr_f, vr_t, vi_f, vi_t) */
            s[1] = col_vr(ly, cs->f_bus[e], r);
            s[2] = col_vr(ly, cs->t_bus[e], r);
            s[3] = col_vi(ly, cs->f_bus[e], r);
            s[4] = col_vi(ly, cs->t_bus[e], r);
        } else {        /* (vm_f, vm_t, va_f, va_t) */
            s[1] = col_vm(ly, cs->f_bus[e], r);
            s[2] = col_vm(ly, cs->t_bus[e], r);
            s[3] = col_va(ly, cs->f_bus[e], r);
            s[4] = col_va(ly, cs->t_bus[e], r);
        }
        break;
    }
    case R_ANG: case R_ANGL:
        if (ly->rect) { /* (vr_f, vr_t, vi_f, vi_t) */
            rw->nsup = 4;
            s[0] = col_vr(ly, cs->f_bus[e], r);
            s[1] = col_vr(ly, cs->t_bus[e], r);
            s[2] = col_vi(ly, cs->f_bus[e], r);
            s[3] = col_vi(ly, cs->t_bus[e], r);
        } else {
            rw->nsup = 2;
            s[0] = col_va(ly, cs->f_bus[e], r);
            s[1] = col_va(ly, cs->t_bus[e], r);
        }
        break;
    case R_BALP: case R_BALQ: {
        int isp = rw->blk == R_BALP;
        int na = adj->arc_ptr[e + 1] - adj->arc_ptr[e];
        int ng = adj->gen_ptr[e + 1] - adj->gen_ptr[e];
        int ns = adj->st_ptr[e + 1] - adj->st_ptr[e];
        const int32_t *dptr = adj->dv_ptr, *didx = adj->dv_idx;
        int nd = dptr[e + 1] - dptr[e];
        rw->nsup = rw->nbv + na + ng + ns + nd;
        rw->narc = na;
        rw->ngen = ng;
        rw->nstor = ns;
        rw->devs = didx + dptr[e];
        if (rw->nsup > (int)(sizeof rw->sup / sizeof rw->sup[0])) {
            rw->big = malloc(sizeof(int64_t) * (size_t)rw->nsup);
            if (!rw->big) return fail("out of memory");
            s = rw->big;
        }
        int q = 0;
        if (ly->rect) {
            s[q++] = col_vr(ly, e, r);
            s[q++] = col_vi(ly, e, r);
        } else {
            s[q++] = col_vm(ly, e, r);
        }
        for (int j = adj->arc_ptr[e]; j < adj->arc_ptr[e + 1]; j++)
            s[q++] = isp ? col_p(ly, adj->arc_idx[j], r) : col_q(ly, adj->arc_idx[j], r);
        for (int j = adj->gen_ptr[e]; j < adj->gen_ptr[e + 1]; j++)
            s[q++] = isp ? col_pg(ly, adj->gen_idx[j], r) : col_qg(ly, adj->gen_idx[j], r);
        for (int j = adj->st_ptr[e]; j < adj->st_ptr[e + 1]; j++)
            s[q++] = isp ? col_ps(ly, adj->st_idx[j], r) : col_qs(ly, adj->st_idx[j], r);
        for (int j = dptr[e]; j < dptr[e + 1]; j++) s[q++] = col_u(ly, didx[j], r);
        break;
    }
    case R_SOC:  /* se_t, se_{t-1} (periods t >= 1), sc_t, sd_t */
        rw->nsup = 0;
        s[rw->nsup++] = col_se(ly, e, r);
        if (r >= 1) s[rw->nsup++] = col_se(ly, e, r - 1);
        s[rw->nsup++] = col_sc(ly, e, r);
        s[rw->nsup++] = col_sd(ly, e, r);
        break;
    case R_SLP:  /* ps, qs, vm of the unit's bus, sd, sc */
        rw->nsup = 5;
        s[0] = col_ps(ly, e, r);
        s[1] = col_qs(ly, e, r);
        s[2] = col_vm(ly, cs->stor_bus[e], r);
        s[3] = col_sd(ly, e, r);
        s[4] = col_sc(ly, e, r);
        break;
    case R_SLQ:  /* ps, qs, vm, qsc */
        rw->nsup = 4;
        s[0] = col_ps(ly, e, r);
        s[1] = col_qs(ly, e, r);
        s[2] = col_vm(ly, cs->stor_bus[e], r);
        s[3] = col_qsc(ly, e, r);
        break;
    case R_STH:  /* ps, qs */
        rw->nsup = 2;
        s[0] = col_ps(ly, e, r);
        s[1] = col_qs(ly, e, r);
        break;
    case R_SCMP: /* sc, sd */
        rw->nsup = 2;
        s[0] = col_sc(ly, e, r);
        s[1] = col_sd(ly, e, r);
        break;
    case R_DRAMP: /* u_t, u_{t-1} */
        rw->nsup = 2;
        s[0] = col_u(ly, e, r);
        s[1] = col_u(ly, e, r - 1);
        break;
    case R_DINIT:
        rw->nsup = 1;
        s[0] = col_u(ly, e, 0);
        break;
    case R_THF: case R_THT: {
        int arc = rw->blk == R_THF ? e : L + e;
        rw->nsup = 2;
        s[0] = col_p(ly, arc, r);
        s[1] = col_q(ly, arc, r);
        break;
    }
    case R_VMAG:
        rw->nsup = 2;
        s[0] = col_vr(ly, e, r);
        s[1] = col_vi(ly, e, r);
        break;
    case R_RAMP:
        rw->nsup = 2;
        s[0] = col_pg(ly, e, r);      /* pg_{k,t} */
        s[1] = col_pg(ly, e, r - 1);  /* pg_{k,t-1} */
        break;
    }
    return 0;
}

/* The terms a balance row adds after its arc terms, in the order of its
 * support: -pg (-qg) of every generator at the bus, +ps (+qs) of every
 * storage unit (the power it draws from the grid), and the device terms
 * cp u (cq u) of every device at the bus (Listing 10 adds the electrolyzer
 * load p_elec to the active balance with constraint!: cp = 1, cq = 0).
 * Devices enter both rows structurally, zero coefficients included. */
static hd balance_tail(const or_case *cs, const row_t *rw, const hd *v, int first, hd acc) {
    int isp = rw->blk == R_BALP;
    int q = first;
    for (int j = 0; j < rw->ngen; j++, q++) acc = hd_sub(acc, v[q]);
    for (int j = 0; j < rw->nstor; j++, q++) acc = hd_add(acc, v[q]);
    for (int j = 0; q < rw->nsup; j++, q++) {
        int d = rw->devs[j];
        acc = hd_add(acc, hd_scale(isp ? cs->dev_cp[d] : cs->dev_cq[d], v[q]));
    }
    return acc;
}

static double bus_pd(const or_case *cs, int i, int r) {
    return (cs->n_periods > 1 && cs->pd_t) ? cs->pd_t[i + (int64_t)cs->n_bus * r] : cs->pd[i];
}
static double bus_qd(const or_case *cs, int i, int r) {
    return (cs->n_periods > 1 && cs->qd_t) ? cs->qd_t[i + (int64_t)cs->n_bus * r] : cs->qd[i];
}

/* The value of one row of the rectangular form (PowerModels' ACR
 * formulation) as a function of its variables v[0..nsup).  With
 * V = vr + j vi the polar terms become polynomials: vm^2 = vr^2 + vi^2,
 * vm_f vm_t cos(th) = vr_f vr_t + vi_f vi_t (CR) and vm_f vm_t sin(th) =
 * vi_f vr_t - vr_f vi_t (SI), so every flow is
 * alpha |V_f|^2 + beta |V_t|^2 + a CR + b SI with the polar coefficients.
 * The angle-difference limits are the two tangent rows
 * SI - tan(angmax) CR <= 0 and SI - tan(angmin) CR >= 0, the voltage
 * magnitude limits the rows vr^2 + vi^2 in [vmin^2, vmax^2], and the
 * reference row fixes vi_r = 0. */
static hd row_value_rect(const or_case *cs, const row_t *rw, const hd *v) {
    int e = rw->ent, r = rw->rep;
    switch (rw->blk) {
    case R_REF:
        return v[0];
    case R_PFR: case R_QFR: case R_PTO: case R_QTO: {
        /* v = (arc variable, vr_f, vr_t, vi_f, vi_t) */
        bcoef k = branch_coef(cs, e, r);
        hd vrf = v[1], vrt = v[2], vif = v[3], vit = v[4];
        hd CR = hd_add(hd_mul(vrf, vrt), hd_mul(vif, vit));
        hd SI = hd_sub(hd_mul(vif, vrt), hd_mul(vrf, vit));
        hd Uf = hd_add(hd_mul(vrf, vrf), hd_mul(vif, vif));
        hd Ut = hd_add(hd_mul(vrt, vrt), hd_mul(vit, vit));
        hd F;
        switch (rw->blk) {
        case R_PFR:
            F = hd_add(hd_scale(k.Gff, Uf), hd_add(hd_scale(k.Gft, CR), hd_scale(k.Bft, SI)));
            break;
        case R_QFR:
            F = hd_add(hd_scale(-k.Bff, Uf), hd_add(hd_scale(-k.Bft, CR), hd_scale(k.Gft, SI)));
            break;
        case R_PTO:
            F = hd_add(hd_scale(k.Gtt, Ut), hd_sub(hd_scale(k.Gtf, CR), hd_scale(k.Btf, SI)));
            break;
        default:
            F = hd_add(hd_scale(-k.Btt, Ut), hd_sub(hd_scale(-k.Btf, CR), hd_scale(k.Gtf, SI)));
            break;
        }
        return hd_sub(v[0], F);
    }
    case R_ANG: case R_ANGL: {
        /* v = (vr_f, vr_t, vi_f, vi_t) */
        double t = tan(rw->blk == R_ANG ? cs->angmax[e] : cs->angmin[e]);
        hd CR = hd_add(hd_mul(v[0], v[1]), hd_mul(v[2], v[3]));
        hd SI = hd_sub(hd_mul(v[2], v[1]), hd_mul(v[0], v[3]));
        return hd_sub(SI, hd_scale(t, CR));
    }
    case R_BALP: case R_BALQ: {
        int isp = rw->blk == R_BALP;
        double load = isp ? bus_pd(cs, e, r) : bus_qd(cs, e, r);
        double shunt = isp ? cs->gs[e] : -cs->bs[e];
        hd v2 = hd_add(hd_mul(v[0], v[0]), hd_mul(v[1], v[1]));
        hd acc = hd_add(hd_cst(load), hd_scale(shunt, v2));
        for (int q = 2; q < 2 + rw->narc; q++) acc = hd_add(acc, v[q]);
        return balance_tail(cs, rw, v, 2 + rw->narc, acc);
    }
    case R_VMAG:
        return hd_add(hd_mul(v[0], v[0]), hd_mul(v[1], v[1]));
    case R_THF: case R_THT: {
        double rate = cs->rate_a[e];
        return hd_sub(hd_add(hd_mul(v[0], v[0]), hd_mul(v[1], v[1])), hd_cst(rate * rate));
    }
    case R_RAMP:
        return hd_sub(v[0], v[1]);
    }
    return hd_cst(NAN);
}

/* The value of one row as a function of its variables v[0..nsup). */
static hd row_value(const or_case *cs, const row_t *rw, const hd *v) {
    int e = rw->ent, r = rw->rep;
    switch (rw->blk) {
    case R_REF:
        return v[0];
    case R_PFR: case R_QFR: case R_PTO: case R_QTO: {
        /* v = (arc variable, vm_f, vm_t, va_f, va_t) */
        bcoef k = branch_coef(cs, e, r);
        hd vmf = v[1], vmt = v[2];
        hd th = hd_sub(v[3], v[4]);
        hd C = hd_cos(th), S = hd_sin(th);
        hd uw = hd_mul(vmf, vmt);
        hd F;
        switch (rw->blk) {
        case R_PFR: /* Re(V_f conj(I_f)) */
            F = hd_add(hd_scale(k.Gff, hd_mul(vmf, vmf)),
                       hd_mul(uw, hd_add(hd_scale(k.Gft, C), hd_scale(k.Bft, S))));
            break;
        case R_QFR: /* Im(V_f conj(I_f)) */
            F = hd_add(hd_scale(-k.Bff, hd_mul(vmf, vmf)),
                       hd_mul(uw, hd_add(hd_scale(-k.Bft, C), hd_scale(k.Gft, S))));
            break;
        case R_PTO: /* Re(V_t conj(I_t)) */
            F = hd_add(hd_scale(k.Gtt, hd_mul(vmt, vmt)),
                       hd_mul(uw, hd_sub(hd_scale(k.Gtf, C), hd_scale(k.Btf, S))));
            break;
        default:    /* Im(V_t conj(I_t)) */
            F = hd_add(hd_scale(-k.Btt, hd_mul(vmt, vmt)),
                       hd_mul(uw, hd_sub(hd_scale(-k.Btf, C), hd_scale(k.Gtf, S))));
            break;
        }
        return hd_sub(v[0], F);
    }
    case R_ANG:
        return hd_sub(v[0], v[1]);
    case R_BALP: case R_BALQ: {
        /* demand and shunt term first, then the terms constraint! adds:
         * +p (+q) of every arc at the bus, -pg (-qg) of every generator */
        int isp = rw->blk == R_BALP;
        double load = isp ? bus_pd(cs, e, r) : bus_qd(cs, e, r);
        double shunt = isp ? cs->gs[e] : -cs->bs[e];
        hd acc = hd_add(hd_cst(load), hd_scale(shunt, hd_mul(v[0], v[0])));
        for (int q = 1; q < 1 + rw->narc; q++) acc = hd_add(acc, v[q]);
        return balance_tail(cs, rw, v, 1 + rw->narc, acc);
    }
    case R_THF: case R_THT: {
        double rate = cs->rate_a[e];
        return hd_sub(hd_add(hd_mul(v[0], v[0]), hd_mul(v[1], v[1])), hd_cst(rate * rate));
    }
    case R_RAMP:
        return hd_sub(v[0], v[1]);
    }
    return hd_cst(NAN);
}

/* Rows of the storage units and the user-extension devices.
 * Storage, per unit u at bus i and period t (the model of Geth, Coffrin and
 * Fobes 2020 that the paper cites for its storage formulation):
 *   state of charge  se_t - se_{t-1} - dt (eta_c sc_t - sd_t / eta_d) = 0,
 *                    se_{-1} = the initial energy e0 (a constant)
 *   active losses    ps + sd - sc - p_loss - r (ps^2 + qs^2) / vm_i^2 = 0
 *   reactive losses  qs - qsc - q_loss - x (ps^2 + qs^2) / vm_i^2 = 0
 *                    ((ps^2 + qs^2) / vm^2 is the squared converter current)
 *   thermal          ps^2 + qs^2 - rating^2 <= 0
 *   complementarity  sc sd <= 0 (with sc, sd >= 0: sc sd = 0), when asked
 * ps, qs: the power the unit draws from the grid (a load in the balance
 * rows); qsc: the converter's reactive set-point; se: stored energy;
 * sc, sd: charging and discharging power.
 * Devices, per device d (Listing 10's electrolyzer generalised to linear
 * devices):  ramp u_t - u_{t-1} (t >= 1) and the initial row u_0. */
static hd row_value_ext(const or_case *cs, const row_t *rw, const hd *v) {
    int e = rw->ent;
    switch (rw->blk) {
    case R_SOC: {
        double dt = cs->stor_dt, ec = cs->stor_eta_c[e], ed = cs->stor_eta_d[e];
        int q = 0;
        hd se = v[q++];
        hd prev = rw->rep >= 1 ? v[q++] : hd_cst(cs->stor_e0[e]);
        hd sc = v[q++], sd = v[q++];
        hd flow = hd_sub(hd_scale(ec, sc), hd_scale(1.0 / ed, sd));
        return hd_sub(hd_sub(se, prev), hd_scale(dt, flow));
    }
    case R_SLP: case R_SLQ: {
        hd ps = v[0], qs = v[1], vm = v[2];
        hd i2 = hd_mul(hd_add(hd_mul(ps, ps), hd_mul(qs, qs)), hd_inv(hd_mul(vm, vm)));
        if (rw->blk == R_SLP) {
            hd sd = v[3], sc = v[4];
            hd lhs = hd_sub(hd_add(ps, sd), sc);
            return hd_sub(hd_sub(lhs, hd_cst(cs->stor_ploss[e])), hd_scale(cs->stor_r[e], i2));
        }
        hd qsc = v[3];
        return hd_sub(hd_sub(hd_sub(qs, qsc), hd_cst(cs->stor_qloss[e])), hd_scale(cs->stor_x[e], i2));
    }
    case R_STH: {
        double rt = cs->stor_rating[e];
        return hd_sub(hd_add(hd_mul(v[0], v[0]), hd_mul(v[1], v[1])), hd_cst(rt * rt));
    }
    case R_SCMP:
        return hd_mul(v[0], v[1]);
    case R_DRAMP:
        return hd_sub(v[0], v[1]);
    case R_DINIT:
        return v[0];
    }
    return hd_cst(NAN);
}

static hd eval_row(const or_case *cs, const row_t *rw, const hd *v) {
    if (rw->blk >= R_SOC) return row_value_ext(cs, rw, v);
    return cs->form ? row_value_rect(cs, rw, v) : row_value(cs, rw, v);
}

/* Hessian support: pairs (i, j) of support positions, i >= j by position
 * order (the caller orders them by column). */
static int row_hess_pairs_rect(const row_t *rw, int pairs[][2]) {
    /* flow rows (positions 1..4 = vr_f, vr_t, vi_f, vi_t): the squares of
     * |V_f|^2 and |V_t|^2, the products of CR and SI; angle rows
     * (positions 0..3): the products of CR and SI */
    static const int flow[8][2] = {{1, 1}, {2, 2}, {3, 3}, {4, 4}, {2, 1}, {4, 3}, {3, 2}, {4, 1}};
    static const int ang[4][2] = {{1, 0}, {3, 2}, {2, 1}, {3, 0}};
    switch (rw->blk) {
    case R_PFR: case R_QFR: case R_PTO: case R_QTO:
        memcpy(pairs, flow, sizeof flow);
        return 8;
    case R_ANG: case R_ANGL:
        memcpy(pairs, ang, sizeof ang);
        return 4;
    case R_BALP: case R_BALQ: case R_VMAG: case R_THF: case R_THT:
        pairs[0][0] = 0; pairs[0][1] = 0;
        pairs[1][0] = 1; pairs[1][1] = 1;
        return 2;
    default:
        return 0;
    }
}

/* Storage and device rows: the loss rows pair ps, qs and vm (positions
 * 0, 1, 2) inside (ps^2 + qs^2) / vm^2 (no ps-qs product), the thermal row
 * squares ps and qs, the complementarity row multiplies sc and sd. */
static int row_hess_pairs_ext(const row_t *rw, int pairs[][2]) {
    static const int loss[5][2] = {{0, 0}, {1, 1}, {2, 2}, {2, 0}, {2, 1}};
    switch (rw->blk) {
    case R_SLP: case R_SLQ:
        memcpy(pairs, loss, sizeof loss);
        return 5;
    case R_STH:
        pairs[0][0] = 0; pairs[0][1] = 0;
        pairs[1][0] = 1; pairs[1][1] = 1;
        return 2;
    case R_SCMP:
        pairs[0][0] = 1; pairs[0][1] = 0;
        return 1;
    default:
        return 0;
    }
}

static int row_hess_pairs(const row_t *rw, int rect, int pairs[][2]) {
    if (rw->blk >= R_SOC) return row_hess_pairs_ext(rw, pairs);
    if (rect) return row_hess_pairs_rect(rw, pairs);
    switch (rw->blk) {
    case R_PFR: case R_QFR: case R_PTO: case R_QTO: {
        int n = 0;
        for (int i = 1; i <= 4; i++)
            for (int j = 1; j <= i; j++) { pairs[n][0] = i; pairs[n][1] = j; n++; }
        return n; /* 10 */
    }
    case R_BALP: case R_BALQ:
        pairs[0][0] = 0; pairs[0][1] = 0;
        return 1;
    case R_THF: case R_THT:
        pairs[0][0] = 0; pairs[0][1] = 0;
        pairs[1][0] = 1; pairs[1][1] = 1;
        return 2;
    default:
        return 0;
    }
}

/* ------------------------------------------------------------------ */
/* row enumeration                                                     */
/* ------------------------------------------------------------------ */
static void row_of(const layout *ly, int64_t row, row_t *rw) {
    int blk = 0;
    while (row >= ly->cblk[blk + 1]) blk++;
    int64_t loc = row - ly->cblk[blk];
    int64_t per;
    switch (blk) {
    case R_REF: per = ly->R; break;
    case R_BALP: case R_BALQ: case R_VMAG: per = ly->N; break;
    case R_RAMP: per = ly->G; break;
    case R_SOC: case R_SLP: case R_SLQ: case R_STH: case R_SCMP: per = ly->S; break;
    case R_DRAMP: case R_DINIT: per = ly->D; break;
    default: per = ly->L; break;
    }
    rw->blk = blk;
    rw->ent = (int)(loc % per);
    rw->rep = (int)(loc / per);
    if (blk == R_RAMP || blk == R_DRAMP) rw->rep += 1; /* ramp rows start at period 1 */
}

/* ------------------------------------------------------------------ */
/* triplets                                                            */
/* ------------------------------------------------------------------ */
typedef struct { int64_t row, col, seq; double val, scale; } trip;
typedef struct { trip *t; int64_t n, cap; } tripvec;

static int tv_push(tripvec *v, int64_t row, int64_t col, double val, double scale) {
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 1024;
        trip *nt = realloc(v->t, sizeof(trip) * (size_t)nc);
        if (!nt) return fail("out of memory");
        v->t = nt; v->cap = nc;
    }
    trip *z = &v->t[v->n];
    z->row = row; z->col = col; z->seq = v->n; z->val = val; z->scale = scale;
    v->n++;
    return 0;
}
static int trip_cmp(const void *pa, const void *pb) {
    const trip *a = pa, *b = pb;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    if (a->seq != b->seq) return a->seq < b->seq ? -1 : 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* validation (only what the oracle itself needs to stay in bounds)   */
/* ------------------------------------------------------------------ */
static int check_case(const or_case *cs) {
    for (int l = 0; l < cs->n_branch; l++) {
        if (cs->f_bus[l] < 0 || cs->f_bus[l] >= cs->n_bus || cs->t_bus[l] < 0 || cs->t_bus[l] >= cs->n_bus)
            return fail("branch bus out of range");
        if (cs->f_bus[l] == cs->t_bus[l]) return fail("branch connects a bus to itself");
    }
    for (int k = 0; k < cs->n_gen; k++)
        if (cs->gen_bus[k] < 0 || cs->gen_bus[k] >= cs->n_bus) return fail("generator bus out of range");
    for (int j = 0; j < cs->n_ref; j++)
        if (cs->ref_bus[j] < 0 || cs->ref_bus[j] >= cs->n_bus) return fail("reference bus out of range");
    for (int s = 0; s < cs->n_cont; s++)
        if (cs->outaged[s] < 0 || cs->outaged[s] >= cs->n_branch) return fail("outaged branch out of range");
    for (int u = 0; u < cs->n_stor; u++)
        if (cs->stor_bus[u] < 0 || cs->stor_bus[u] >= cs->n_bus) return fail("storage bus out of range");
    for (int d = 0; d < cs->n_dev; d++)
        if (cs->dev_bus[d] < 0 || cs->dev_bus[d] >= cs->n_bus) return fail("device bus out of range");
    return 0;
}

int or_dims(const or_case *cs, int64_t *n, int64_t *m) {
    layout ly;
    if (make_layout(cs, &ly)) return -1;
    *n = ly.n;
    *m = ly.cblk[R_NBLK];
    return 0;
}

/* ------------------------------------------------------------------ */
/* bounds and starting point                                           */
/* ------------------------------------------------------------------ */
int or_bounds(const or_case *cs, double *lvar, double *uvar, double *lcon, double *ucon, double *x0) {
    layout ly;
    if (make_layout(cs, &ly) || check_case(cs)) return -1;
    int N = ly.N, L = ly.L, G = ly.G;
    for (int64_t j = 0; j < ly.n; j++) { lvar[j] = -INFINITY; uvar[j] = INFINITY; x0[j] = 0.0; }
    for (int r = 0; r < ly.nrep; r++) {
        for (int i = 0; i < N; i++) {
            if (ly.rect) {
                /* |vr|, |vi| <= vmax; start vr = 1, vi = 0 */
                int64_t cr = col_vr(&ly, i, r), ci = col_vi(&ly, i, r);
                lvar[cr] = -cs->vmax[i]; uvar[cr] = cs->vmax[i]; x0[cr] = 1.0;
                lvar[ci] = -cs->vmax[i]; uvar[ci] = cs->vmax[i];
            } else {
                int64_t c = col_vm(&ly, i, r);
                lvar[c] = cs->vmin[i]; uvar[c] = cs->vmax[i]; x0[c] = 1.0;
            }
        }
        for (int k = 0; k < G; k++) {
            if (r < ly.npg) { int64_t c = col_pg(&ly, k, r); lvar[c] = cs->pmin[k]; uvar[c] = cs->pmax[k]; }
            int64_t c = col_qg(&ly, k, r);
            lvar[c] = cs->qmin[k]; uvar[c] = cs->qmax[k];
        }
        for (int a = 0; a < 2 * L; a++) {
            double rate = cs->rate_a[a < L ? a : a - L];
            lvar[col_p(&ly, a, r)] = -rate; uvar[col_p(&ly, a, r)] = rate;
            lvar[col_q(&ly, a, r)] = -rate; uvar[col_q(&ly, a, r)] = rate;
        }
        for (int u = 0; u < ly.S; u++) {
            double rt = cs->stor_rating[u];
            lvar[col_ps(&ly, u, r)] = -rt; uvar[col_ps(&ly, u, r)] = rt;
            lvar[col_qs(&ly, u, r)] = cs->stor_qmin[u]; uvar[col_qs(&ly, u, r)] = cs->stor_qmax[u];
            lvar[col_qsc(&ly, u, r)] = -rt; uvar[col_qsc(&ly, u, r)] = rt;
            lvar[col_se(&ly, u, r)] = 0.0; uvar[col_se(&ly, u, r)] = cs->stor_emax[u];
            lvar[col_sc(&ly, u, r)] = 0.0; uvar[col_sc(&ly, u, r)] = cs->stor_chmax[u];
            lvar[col_sd(&ly, u, r)] = 0.0; uvar[col_sd(&ly, u, r)] = cs->stor_dismax[u];
        }
        for (int d = 0; d < ly.D; d++) {
            lvar[col_u(&ly, d, r)] = cs->dev_lo[d]; uvar[col_u(&ly, d, r)] = cs->dev_hi[d];
        }
    }
    int64_t m = ly.cblk[R_NBLK];
    for (int64_t row = 0; row < m; row++) {
        row_t rw;
        row_of(&ly, row, &rw);
        double lo = 0.0, hi = 0.0;
        int out = (rw.blk == R_ANG || rw.blk == R_ANGL) && cs->n_cont > 0 && rw.rep >= 1 &&
                  cs->outaged[rw.rep - 1] == rw.ent;
        if (out) {
            lo = -INFINITY; hi = INFINITY;
        } else if (rw.blk == R_ANG && !ly.rect) {
            lo = cs->angmin[rw.ent]; hi = cs->angmax[rw.ent];
        } else if (rw.blk == R_ANG) {   /* SI - tan(angmax) CR <= 0 */
            lo = -INFINITY; hi = 0.0;
        } else if (rw.blk == R_ANGL) {  /* SI - tan(angmin) CR >= 0 */
            lo = 0.0; hi = INFINITY;
        } else if (rw.blk == R_VMAG) {
            lo = cs->vmin[rw.ent] * cs->vmin[rw.ent];
            hi = cs->vmax[rw.ent] * cs->vmax[rw.ent];
        } else if (rw.blk == R_THF || rw.blk == R_THT) {
            lo = -INFINITY; hi = 0.0;
        } else if (rw.blk == R_RAMP) {
            lo = -cs->ramp_ratio * cs->pmax[rw.ent];
            hi = cs->ramp_ratio * cs->pmax[rw.ent];
        } else if (rw.blk == R_STH || rw.blk == R_SCMP) {
            lo = -INFINITY; hi = 0.0;
        } else if (rw.blk == R_DRAMP) {
            lo = -cs->dev_ramp[rw.ent]; hi = cs->dev_ramp[rw.ent];
        } else if (rw.blk == R_DINIT) {
            lo = cs->dev_init_lo[rw.ent]; hi = cs->dev_init_hi[rw.ent];
        }
        lcon[row] = lo; ucon[row] = hi;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* evaluation                                                          */
/* ------------------------------------------------------------------ */
enum { W_OBJ = 1, W_CONS = 2, W_JAC = 4, W_HESS = 8 };

void or_free(or_result *res) {
    if (!res) return;
    free(res->g); free(res->c); free(res->cscale);
    free(res->jrow); free(res->jcol); free(res->jval); free(res->jscale);
    free(res->hrow); free(res->hcol); free(res->hval); free(res->hscale);
    free(res);
}

/* Evaluate a row on seeded hyper-duals: seeds at support positions s1, s2
 * (-1 = none).  s1 == s2 seeds both directions on the same variable. */
static hd seeded(const or_case *cs, const row_t *rw, const double *x,
                 hd *buf, int s1, int s2) {
    const int64_t *sup = row_sup((row_t *)rw);
    for (int q = 0; q < rw->nsup; q++)
        buf[q] = hd_var(x[sup[q]], q == s1 ? 1.0 : 0.0, q == s2 ? 1.0 : 0.0);
    return eval_row(cs, rw, buf);
}

or_result *or_eval(const or_case *cs, const double *x, const double *y, double sigma, int want) {
    layout ly;
    if (make_layout(cs, &ly) || check_case(cs)) return NULL;
    adjacency adj;
    memset(&adj, 0, sizeof adj);
    if (build_adjacency(cs, &adj)) { free_adjacency(&adj); return NULL; }
    or_result *res = calloc(1, sizeof *res);
    if (!res) { free_adjacency(&adj); fail("out of memory"); return NULL; }
    int64_t n = ly.n, m = ly.cblk[R_NBLK];
    res->n = n; res->m = m;
    int maxsup = 1;
    for (int i = 0; i < ly.N; i++) {
        int s = 2 + (adj.arc_ptr[i + 1] - adj.arc_ptr[i]) + (adj.gen_ptr[i + 1] - adj.gen_ptr[i]) +
                (adj.st_ptr[i + 1] - adj.st_ptr[i]) + (adj.dv_ptr[i + 1] - adj.dv_ptr[i]);
        if (s > maxsup) maxsup = s;
    }
    if (maxsup < 5) maxsup = 5;
    hd *buf = malloc(sizeof(hd) * (size_t)maxsup);
    tripvec J = {0}, H = {0};
    int err = 0;
    if (!buf) { fail("out of memory"); err = 1; goto done; }

    /* objective, gradient and the objective's Hessian terms (the pg block) */
    if (want & (W_OBJ | W_HESS)) {
        res->g = calloc((size_t)n, sizeof(double));
        if (!res->g) { fail("out of memory"); err = 1; goto done; }
        double f = 0.0, fs = 0.0;
        for (int r = 0; r < ly.npg; r++) {
            for (int k = 0; k < ly.G; k++) {
                int64_t col = col_pg(&ly, k, r);
                hd pg = hd_var(x[col], 1.0, 1.0);
                hd term = hd_add(hd_add(hd_scale(cs->c2[k], hd_mul(pg, pg)), hd_scale(cs->c1[k], pg)),
                                 hd_cst(cs->c0[k]));
                f += term.a;
                fs += term.ma;
                res->g[col] = term.b;
                if (want & W_HESS)
                    if (tv_push(&H, col, col, sigma * term.d, fabs(sigma) * term.md)) { err = 1; goto done; }
            }
        }
        /* the devices' secondary objective (Listing 10): cost_d u_{d,t} */
        for (int r = 0; r < ly.nrep; r++)
            for (int d = 0; d < ly.D; d++) {
                int64_t col = col_u(&ly, d, r);
                hd term = hd_scale(cs->dev_cost[d], hd_var(x[col], 1.0, 1.0));
                f += term.a;
                fs += term.ma;
                res->g[col] = term.b;
            }
        res->f = f;
        res->fscale = fs;
    }

    if (want & (W_CONS | W_JAC | W_HESS)) {
        if (want & W_CONS) {
            res->c = malloc(sizeof(double) * (size_t)(m ? m : 1));
            res->cscale = malloc(sizeof(double) * (size_t)(m ? m : 1));
            if (!res->c || !res->cscale) { fail("out of memory"); err = 1; goto done; }
        }
        for (int64_t row = 0; row < m; row++) {
            row_t rw;
            row_of(&ly, row, &rw);
            if (row_support(cs, &ly, &adj, &rw)) { err = 1; goto done; }
            const int64_t *sup = row_sup(&rw);
            if (want & W_CONS) {
                hd v = seeded(cs, &rw, x, buf, -1, -1);
                res->c[row] = v.a;
                res->cscale[row] = v.ma;
            }
            if (want & W_JAC) {
                for (int q = 0; q < rw.nsup; q++) {
                    hd v = seeded(cs, &rw, x, buf, q, -1);
                    if (tv_push(&J, row, sup[q], v.b, v.mb)) { err = 1; goto done; }
                }
            }
            if (want & W_HESS) {
                int pairs[16][2];
                int np = row_hess_pairs(&rw, ly.rect, pairs);
                for (int p = 0; p < np; p++) {
                    int s1 = pairs[p][0], s2 = pairs[p][1];
                    hd v = seeded(cs, &rw, x, buf, s1, s2);
                    int64_t c1 = sup[s1], c2 = sup[s2];
                    int64_t hr = c1 > c2 ? c1 : c2, hc = c1 > c2 ? c2 : c1;
                    if (tv_push(&H, hr, hc, y[row] * v.d, fabs(y[row]) * v.md)) { err = 1; goto done; }
                }
            }
            free(rw.big);
        }
    }

    if (want & W_JAC) {
        /* rows are emitted in order; sort each row's entries by column */
        qsort(J.t, (size_t)J.n, sizeof(trip), trip_cmp);
        res->nnzj = J.n;
        res->jrow = malloc(sizeof(int32_t) * (size_t)(J.n + 1));
        res->jcol = malloc(sizeof(int32_t) * (size_t)(J.n + 1));
        res->jval = malloc(sizeof(double) * (size_t)(J.n + 1));
        res->jscale = malloc(sizeof(double) * (size_t)(J.n + 1));
        if (!res->jrow || !res->jcol || !res->jval || !res->jscale) { fail("out of memory"); err = 1; goto done; }
        for (int64_t e = 0; e < J.n; e++) {
            if (e > 0 && J.t[e].row == J.t[e - 1].row && J.t[e].col == J.t[e - 1].col) {
                fail("duplicate Jacobian entry");
                err = 1;
                goto done;
            }
            res->jrow[e] = (int32_t)J.t[e].row;
            res->jcol[e] = (int32_t)J.t[e].col;
            res->jval[e] = J.t[e].val;
            res->jscale[e] = J.t[e].scale;
        }
    }
    if (want & W_HESS) {
        /* stable by emission order: objective first, then rows ascending */
        qsort(H.t, (size_t)H.n, sizeof(trip), trip_cmp);
        int64_t u = 0;
        for (int64_t e = 0; e < H.n; e++) {
            if (u > 0 && H.t[u - 1].row == H.t[e].row && H.t[u - 1].col == H.t[e].col) {
                H.t[u - 1].val += H.t[e].val;
                H.t[u - 1].scale += H.t[e].scale;
            } else {
                H.t[u++] = H.t[e];
            }
        }
        res->nnzh = u;
        res->hrow = malloc(sizeof(int32_t) * (size_t)(u + 1));
        res->hcol = malloc(sizeof(int32_t) * (size_t)(u + 1));
        res->hval = malloc(sizeof(double) * (size_t)(u + 1));
        res->hscale = malloc(sizeof(double) * (size_t)(u + 1));
        if (!res->hrow || !res->hcol || !res->hval || !res->hscale) { fail("out of memory"); err = 1; goto done; }
        for (int64_t e = 0; e < u; e++) {
            res->hrow[e] = (int32_t)H.t[e].row;
            res->hcol[e] = (int32_t)H.t[e].col;
            res->hval[e] = H.t[e].val;
            res->hscale[e] = H.t[e].scale;
        }
    }

done:
    free(buf);
    free(J.t);
    free(H.t);
    free_adjacency(&adj);
    if (err) { or_free(res); return NULL; }
    return res;
}
