// Host-side model construction (see host_model.h).  The rule below is the
// polar form's; the rectangular form's (bus blocks vr, vi) follows it in
// fill_pattern.
//
// Pattern rule (structural, 0-based, sorted by (row, col), unique):
//  Jacobian, rows in constraint order:
//   ref        [va_r]
//   flow row   [va_lo, va_hi, vm_lo, vm_hi, arc variable]   lo/hi = min/max(f, t)
//   angle      [va_lo, va_hi]
//   balance    [vm_i, generator columns ascending, arc columns ascending]
//   thermal    [p_a, q_a]
//   ramp       [pg_{k,t-1}, pg_{k,t}]
//  Hessian lower triangle, per replica:
//   va row i   [va_k for distinct neighbours k < i], va_i      (if i has a branch)
//   vm row i   [va_k for distinct neighbours k < i], va_i, [va_k for k > i],
//              [vm_k for distinct neighbours k < i], vm_i       (if i has a branch)
//              vm_i only                                        (isolated bus)
//   pg row     diagonal (objective), p row and q row: diagonal (thermal)
//  These are exactly the variable pairs that share a nonlinear term: the four
//  voltage variables of a branch's flow rows, vm^2 of the balance shunt term,
//  p^2 and q^2 of a thermal row, pg^2 of a cost term.
#include "host_model.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>

namespace opf {

namespace {

int fail(std::string& err, int code, const char* fmt, long long a = 0, long long b = 0) {
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, a, b);
    err = buf;
    return code;
}

int32_t nperiods(const opf_opts* o) { return o ? o->n_periods : 1; }
int32_t ncont(const opf_opts* o) { return o ? o->n_cont : 0; }
int32_t form(const opf_opts* o) { return o ? o->form : OPF_FORM_POLAR; }
int32_t nstor(const opf_opts* o) { return (o && o->storage) ? o->storage->n : 0; }
int32_t ndev(const opf_opts* o) { return (o && o->devices) ? o->devices->n : 0; }

}  // namespace

int validate(const opf_case* cs, const opf_opts* opts, std::string& err) {
    if (!cs) return fail(err, OPF_E_ARG, "case is NULL");
    if (cs->n_bus < 1) return fail(err, OPF_E_CASE, "n_bus must be >= 1 (got %lld)", cs->n_bus);
    if (cs->n_branch < 0 || cs->n_gen < 0) return fail(err, OPF_E_CASE, "negative branch or generator count");
    if (cs->n_ref < 1) return fail(err, OPF_E_CASE, "at least one reference bus is required");
    const int32_t N = cs->n_bus, L = cs->n_branch, G = cs->n_gen;
    if (!cs->pd || !cs->qd || !cs->gs || !cs->bs || !cs->vmin || !cs->vmax || !cs->ref_bus)
        return fail(err, OPF_E_ARG, "a bus array is NULL");
    if (L > 0 && (!cs->f_bus || !cs->t_bus || !cs->r || !cs->x || !cs->b || !cs->tap || !cs->shift ||
                  !cs->rate_a || !cs->angmin || !cs->angmax))
        return fail(err, OPF_E_ARG, "a branch array is NULL");
    if (G > 0 && (!cs->gen_bus || !cs->pmin || !cs->pmax || !cs->qmin || !cs->qmax || !cs->c2 || !cs->c1 ||
                  !cs->c0))
        return fail(err, OPF_E_ARG, "a generator array is NULL");
    for (int32_t j = 0; j < cs->n_ref; j++)
        if (cs->ref_bus[j] < 0 || cs->ref_bus[j] >= N)
            return fail(err, OPF_E_CASE, "reference %lld names bus %lld, out of range", j, cs->ref_bus[j]);
    for (int32_t i = 0; i < N; i++)
        if (!(cs->vmin[i] <= cs->vmax[i])) return fail(err, OPF_E_CASE, "bus %lld has vmin > vmax", i);
    std::vector<int32_t> deg(N, 0);
    for (int32_t l = 0; l < L; l++) {
        int32_t f = cs->f_bus[l], t = cs->t_bus[l];
        if (f < 0 || f >= N || t < 0 || t >= N)
            return fail(err, OPF_E_CASE, "branch %lld has a bus out of range", l);
        if (f == t) return fail(err, OPF_E_CASE, "branch %lld connects bus %lld to itself", l, f);
        double z = cs->r[l] * cs->r[l] + cs->x[l] * cs->x[l];
        if (!(z > 0.0) || !std::isfinite(z)) return fail(err, OPF_E_CASE, "branch %lld has zero impedance", l);
        if (!(cs->tap[l] > 0.0) || !std::isfinite(cs->tap[l]))
            return fail(err, OPF_E_CASE, "branch %lld has a nonpositive tap ratio", l);
        if (!std::isfinite(cs->shift[l]) || !std::isfinite(cs->b[l]) || !std::isfinite(cs->rate_a[l]))
            return fail(err, OPF_E_CASE, "branch %lld has a non-finite parameter", l);
        if (++deg[f] > OPF_MAX_DEGREE || ++deg[t] > OPF_MAX_DEGREE)
            return fail(err, OPF_E_CASE, "branch %lld takes a bus past %lld branches", l, OPF_MAX_DEGREE);
    }
    for (int32_t k = 0; k < G; k++) {
        if (cs->gen_bus[k] < 0 || cs->gen_bus[k] >= N)
            return fail(err, OPF_E_CASE, "generator %lld has a bus out of range", k);
        if (!(cs->pmin[k] <= cs->pmax[k])) return fail(err, OPF_E_CASE, "generator %lld has pmin > pmax", k);
        if (!(cs->qmin[k] <= cs->qmax[k])) return fail(err, OPF_E_CASE, "generator %lld has qmin > qmax", k);
    }
    const int32_t T = nperiods(opts), K = ncont(opts);
    if (T < 1) return fail(err, OPF_E_CASE, "n_periods must be >= 1 (got %lld)", T);
    if (K < 0) return fail(err, OPF_E_CASE, "n_cont must be >= 0 (got %lld)", K);
    if (T > 1 && K > 0) return fail(err, OPF_E_CASE, "periods and contingency copies cannot be combined");
    if (form(opts) != OPF_FORM_POLAR && form(opts) != OPF_FORM_RECT)
        return fail(err, OPF_E_CASE, "form must be OPF_FORM_POLAR or OPF_FORM_RECT (got %lld)", form(opts));
    if (opts && T > 1 && (!(opts->ramp_ratio >= 0.0) || !std::isfinite(opts->ramp_ratio)))
        return fail(err, OPF_E_CASE, "ramp_ratio must be finite and >= 0");
    if (opts && (opts->pd_t == nullptr) != (opts->qd_t == nullptr))
        return fail(err, OPF_E_ARG, "pd_t and qd_t must both be given or both be NULL");
    if (K > 0) {
        if (!opts->outaged_branch) return fail(err, OPF_E_ARG, "outaged_branch is NULL");
        for (int32_t s = 0; s < K; s++)
            if (opts->outaged_branch[s] < 0 || opts->outaged_branch[s] >= L)
                return fail(err, OPF_E_CASE, "contingency %lld outages branch %lld, out of range", s,
                            opts->outaged_branch[s]);
    }
    const int32_t S = nstor(opts), D = ndev(opts);
    if (S < 0 || D < 0) return fail(err, OPF_E_CASE, "negative storage or device count");
    if ((S > 0 || D > 0) && K > 0)
        return fail(err, OPF_E_CASE, "storage units and devices cannot be combined with contingency copies");
    if (S > 0) {
        const opf_storage* st = opts->storage;
        if (form(opts) != OPF_FORM_POLAR) return fail(err, OPF_E_CASE, "storage units take the polar form");
        if (!st->bus || !st->emax || !st->chmax || !st->dismax || !st->rating || !st->qmin || !st->qmax ||
            !st->eta_c || !st->eta_d || !st->r || !st->x || !st->ploss || !st->qloss || !st->e0)
            return fail(err, OPF_E_ARG, "a storage array is NULL");
        if (!(st->dt > 0.0) || !std::isfinite(st->dt)) return fail(err, OPF_E_CASE, "storage dt must be > 0");
        for (int32_t u = 0; u < S; u++) {
            if (st->bus[u] < 0 || st->bus[u] >= N)
                return fail(err, OPF_E_CASE, "storage unit %lld has a bus out of range", u);
            if (!(st->eta_c[u] > 0.0) || !(st->eta_d[u] > 0.0))
                return fail(err, OPF_E_CASE, "storage unit %lld has a nonpositive efficiency", u);
            if (!(st->qmin[u] <= st->qmax[u]) || !(st->emax[u] >= 0.0) || !(st->chmax[u] >= 0.0) ||
                !(st->dismax[u] >= 0.0) || !(st->rating[u] >= 0.0))
                return fail(err, OPF_E_CASE, "storage unit %lld has inconsistent ratings", u);
        }
    }
    if (D > 0) {
        const opf_devices* dv = opts->devices;
        if (!dv->bus || !dv->cp || !dv->cq || !dv->cost || !dv->lo || !dv->hi || !dv->ramp || !dv->init_lo ||
            !dv->init_hi)
            return fail(err, OPF_E_ARG, "a device array is NULL");
        for (int32_t d = 0; d < D; d++) {
            if (dv->bus[d] < 0 || dv->bus[d] >= N)
                return fail(err, OPF_E_CASE, "device %lld has a bus out of range", d);
            if (!(dv->lo[d] <= dv->hi[d]) || !(dv->init_lo[d] <= dv->init_hi[d]))
                return fail(err, OPF_E_CASE, "device %lld has lo > hi", d);
        }
    }
    // sizes must fit the int32 pattern indices
    const int64_t nrep = T > 1 ? T : (int64_t)K + 1;
    const int64_t npg = K > 0 ? 1 : nrep;
    const int64_t n = nrep * (2LL * N + G + 4LL * L + 6LL * S + D) + npg * G;
    const bool rect = form(opts) == OPF_FORM_RECT;
    const int64_t m = nrep * (cs->n_ref + (rect ? 8LL : 7LL) * L + (rect ? 3LL : 2LL) * N) +
                      (T > 1 ? (int64_t)G * (T - 1) : 0);
    const int64_t nnzj = nrep * (cs->n_ref + (rect ? 36LL : 30LL) * L + (rect ? 6LL : 2LL) * N + 2LL * G) +
                         2LL * G * (T - 1) + nrep * (19LL * S + 2LL * D) + 2LL * D * (T - 1) + D;
    const int64_t lim = std::numeric_limits<int32_t>::max();
    if (n >= lim || m >= lim || nnzj >= lim) return fail(err, OPF_E_CASE, "model too large for int32 indices");
    return OPF_OK;
}

int build_host_model(const opf_case* cs, const opf_opts* opts, HostModel& hm, std::string& err) {
    int rc = validate(cs, opts, err);
    if (rc) return rc;
    const int32_t N = cs->n_bus, L = cs->n_branch, G = cs->n_gen, R = cs->n_ref;
    const int32_t T = nperiods(opts), K = ncont(opts);
    Layout& ly = hm.ly;
    ly.N = N; ly.L = L; ly.G = G; ly.R = R; ly.T = T; ly.K = K;
    ly.nrep = T > 1 ? T : K + 1;
    ly.npg = K > 0 ? 1 : ly.nrep;
    ly.rect = form(opts) == OPF_FORM_RECT ? 1 : 0;
    const int64_t P = ly.nrep;

    // ---- branch terms of the pi model (series g + jb, charging b/2 a side,
    // ideal transformer tr + j ti on the from side)
    hm.f_bus.assign(cs->f_bus, cs->f_bus + L);
    hm.t_bus.assign(cs->t_bus, cs->t_bus + L);
    hm.coef.assign(8 * (size_t)L, 0.0);
    hm.rate2.resize(L);
    for (int32_t l = 0; l < L; l++) {
        const double z = cs->r[l] * cs->r[l] + cs->x[l] * cs->x[l];
        const double g = cs->r[l] / z, b = -cs->x[l] / z;
        const double tr = cs->tap[l] * std::cos(cs->shift[l]);
        const double ti = cs->tap[l] * std::sin(cs->shift[l]);
        const double t2 = cs->tap[l] * cs->tap[l];
        const double bc = 0.5 * cs->b[l];
        double* k = hm.coef.data();
        k[0 * (size_t)L + l] = g / t2;                     // Gff
        k[1 * (size_t)L + l] = (b + bc) / t2;              // Bff
        k[2 * (size_t)L + l] = (-g * tr + b * ti) / t2;    // Gft
        k[3 * (size_t)L + l] = (-b * tr - g * ti) / t2;    // Bft
        k[4 * (size_t)L + l] = g;                          // Gtt
        k[5 * (size_t)L + l] = b + bc;                     // Btt
        k[6 * (size_t)L + l] = (-g * tr - b * ti) / t2;    // Gtf
        k[7 * (size_t)L + l] = (-b * tr + g * ti) / t2;    // Btf
        hm.rate2[l] = cs->rate_a[l] * cs->rate_a[l];
    }
    if (ly.rect) {
        hm.tan_lim.resize(2 * (size_t)L);
        for (int32_t l = 0; l < L; l++) {
            hm.tan_lim[l] = std::tan(cs->angmax[l]);
            hm.tan_lim[(size_t)L + l] = std::tan(cs->angmin[l]);
        }
    }

    // ---- half-edges per bus, sorted by (neighbour, branch)
    hm.adj_ptr.assign(N + 1, 0);
    for (int32_t l = 0; l < L; l++) {
        hm.adj_ptr[cs->f_bus[l] + 1]++;
        hm.adj_ptr[cs->t_bus[l] + 1]++;
    }
    for (int32_t i = 0; i < N; i++) hm.adj_ptr[i + 1] += hm.adj_ptr[i];
    hm.he.resize(2 * (size_t)L);
    {
        std::vector<int32_t> fill(hm.adj_ptr.begin(), hm.adj_ptr.end() - 1);
        for (int32_t l = 0; l < L; l++) {
            hm.he[fill[cs->f_bus[l]]++] = (l << 1) | 1;
            hm.he[fill[cs->t_bus[l]]++] = (l << 1);
        }
    }
    auto nbr = [&](int32_t code) {
        const int32_t l = code >> 1;
        return (code & 1) ? cs->t_bus[l] : cs->f_bus[l];
    };
    hm.he_grp.resize(2 * (size_t)L);
    hm.nlo.assign(N, 0);
    hm.ndist.assign(N, 0);
    hm.max_degree = 0;
    for (int32_t i = 0; i < N; i++) {
        auto b = hm.he.begin() + hm.adj_ptr[i], e = hm.he.begin() + hm.adj_ptr[i + 1];
        std::sort(b, e, [&](int32_t u, int32_t v) {
            const int32_t nu = nbr(u), nv = nbr(v);
            return nu != nv ? nu < nv : (u >> 1) < (v >> 1);
        });
        int32_t grp = -1, prev = -1;
        for (int32_t q = hm.adj_ptr[i]; q < hm.adj_ptr[i + 1]; q++) {
            const int32_t k = nbr(hm.he[q]);
            if (k != prev) {
                grp++;
                prev = k;
                if (k < i) hm.nlo[i]++;
            }
            hm.he_grp[q] = grp;
        }
        hm.ndist[i] = grp + 1;
        hm.max_degree = std::max(hm.max_degree, hm.adj_ptr[i + 1] - hm.adj_ptr[i]);
    }

    // ---- generators and arcs per bus (ascending index)
    hm.gen_ptr.assign(N + 1, 0);
    for (int32_t k = 0; k < G; k++) hm.gen_ptr[cs->gen_bus[k] + 1]++;
    for (int32_t i = 0; i < N; i++) hm.gen_ptr[i + 1] += hm.gen_ptr[i];
    hm.gen_list.resize(G);
    {
        std::vector<int32_t> fill(hm.gen_ptr.begin(), hm.gen_ptr.end() - 1);
        for (int32_t k = 0; k < G; k++) hm.gen_list[fill[cs->gen_bus[k]]++] = k;
    }
    hm.arc_ptr.assign(N + 1, 0);
    for (int32_t a = 0; a < 2 * L; a++) hm.arc_ptr[(a < L ? cs->f_bus[a] : cs->t_bus[a - L]) + 1]++;
    for (int32_t i = 0; i < N; i++) hm.arc_ptr[i + 1] += hm.arc_ptr[i];
    hm.arc_list.resize(2 * (size_t)L);
    {
        std::vector<int32_t> fill(hm.arc_ptr.begin(), hm.arc_ptr.end() - 1);
        for (int32_t a = 0; a < 2 * L; a++) hm.arc_list[fill[a < L ? cs->f_bus[a] : cs->t_bus[a - L]]++] = a;
    }

    // ---- per-bus offsets of the balance Jacobian rows and Hessian bus rows
    hm.jbal_off.assign(N + 1, 0);
    hm.hva_off.assign(N + 1, 0);
    hm.hvm_off.assign(N + 1, 0);
    for (int32_t i = 0; i < N; i++) {
        const int32_t deg = hm.adj_ptr[i + 1] - hm.adj_ptr[i];
        const int32_t ng = hm.gen_ptr[i + 1] - hm.gen_ptr[i];
        if (ly.rect) {
            // balance rows lead with vr_i, vi_i; the vr row holds (vr_i, vr_k)
            // for k < i and the diagonal, the vi row (vi_i, vr_k) for every
            // neighbour, (vi_i, vi_k) for k < i and the diagonal (no
            // (vi_i, vr_i) term exists)
            hm.jbal_off[i + 1] = hm.jbal_off[i] + 2 + ng + deg;
            hm.hva_off[i + 1] = hm.hva_off[i] + hm.nlo[i] + 1;
            hm.hvm_off[i + 1] = hm.hvm_off[i] + hm.ndist[i] + hm.nlo[i] + 1;
        } else {
            hm.jbal_off[i + 1] = hm.jbal_off[i] + 1 + ng + deg;
            hm.hva_off[i + 1] = hm.hva_off[i] + (deg > 0 ? hm.nlo[i] + 1 : 0);
            hm.hvm_off[i + 1] = hm.hvm_off[i] + (deg > 0 ? hm.ndist[i] + hm.nlo[i] + 2 : 1);
        }
    }

    // ---- bus, generator and replica data
    hm.gs.assign(cs->gs, cs->gs + N);
    hm.bs.assign(cs->bs, cs->bs + N);
    if (T > 1 && opts && opts->pd_t) {
        hm.pd.assign(opts->pd_t, opts->pd_t + (size_t)N * T);
        hm.qd.assign(opts->qd_t, opts->qd_t + (size_t)N * T);
        hm.load_stride = N;
    } else {
        hm.pd.assign(cs->pd, cs->pd + N);
        hm.qd.assign(cs->qd, cs->qd + N);
        hm.load_stride = 0;
    }
    hm.c2.assign(cs->c2, cs->c2 + G);
    hm.c1.assign(cs->c1, cs->c1 + G);
    hm.c0.assign(cs->c0, cs->c0 + G);
    hm.gen_bus.assign(cs->gen_bus, cs->gen_bus + G);
    hm.ref_bus.assign(cs->ref_bus, cs->ref_bus + R);
    hm.ref_ptr.assign(N + 1, 0);
    for (int32_t j = 0; j < R; j++) hm.ref_ptr[cs->ref_bus[j] + 1]++;
    for (int32_t i = 0; i < N; i++) hm.ref_ptr[i + 1] += hm.ref_ptr[i];
    hm.ref_list.resize(R);
    hm.is_ref.assign(N, 0);
    for (int32_t j = 0; j < R; j++) hm.is_ref[cs->ref_bus[j]] = 1;
    {
        std::vector<int32_t> fill(hm.ref_ptr.begin(), hm.ref_ptr.end() - 1);
        for (int32_t j = 0; j < R; j++) hm.ref_list[fill[cs->ref_bus[j]]++] = j;
    }
    hm.outage.assign(P, -1);
    for (int32_t s = 0; s < K; s++) hm.outage[s + 1] = opts->outaged_branch[s];

    // ---- storage units and devices
    const int32_t S = nstor(opts), D = ndev(opts);
    ly.S = S;
    ly.D = D;
    ly.comp = (S > 0 && opts->storage->comp) ? 1 : 0;
    auto per_bus = [&](int32_t count, const std::vector<int32_t>& bus, std::vector<int32_t>& ptr,
                       std::vector<int32_t>& list) {
        ptr.assign(N + 1, 0);
        for (int32_t e = 0; e < count; e++) ptr[bus[e] + 1]++;
        for (int32_t i = 0; i < N; i++) ptr[i + 1] += ptr[i];
        list.resize(count);
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int32_t e = 0; e < count; e++) list[fill[bus[e]]++] = e;
    };
    if (S > 0) {
        const opf_storage* st = opts->storage;
        hm.stor_bus.assign(st->bus, st->bus + S);
        const double* par[kStorPar] = {st->emax, st->chmax, st->dismax, st->rating, st->qmin, st->qmax, st->eta_c,
                                       st->eta_d, st->r, st->x, st->ploss, st->qloss, st->e0};
        hm.stor_par.resize((size_t)kStorPar * S);
        for (int k = 0; k < kStorPar; k++)
            std::copy(par[k], par[k] + S, hm.stor_par.begin() + (size_t)k * S);
        hm.stor_dt = st->dt;
    }
    if (D > 0) {
        const opf_devices* dv = opts->devices;
        hm.dev_bus.assign(dv->bus, dv->bus + D);
        const double* par[kDevPar] = {dv->cp, dv->cq, dv->cost};
        hm.dev_par.resize((size_t)kDevPar * D);
        for (int k = 0; k < kDevPar; k++) std::copy(par[k], par[k] + D, hm.dev_par.begin() + (size_t)k * D);
    }
    per_bus(S, hm.stor_bus, hm.st_ptr, hm.st_list);
    per_bus(D, hm.dev_bus, hm.dv_ptr, hm.dv_list);
    // balance rows also hold one entry per storage unit and device at the bus
    for (int32_t i = N - 1; i >= 0; i--) {
        const int32_t extra = (hm.st_ptr[i + 1] + hm.dv_ptr[i + 1]);
        hm.jbal_off[i + 1] += extra;
    }

    // ---- layout
    ly.x_va = 0;
    ly.x_vm = N * P;
    ly.x_pg = 2LL * N * P;
    ly.x_qg = ly.x_pg + (int64_t)G * ly.npg;
    ly.x_p = ly.x_qg + (int64_t)G * P;
    ly.x_q = ly.x_p + 2LL * L * P;
    ly.x_ps = ly.x_q + 2LL * L * P;
    ly.x_qs = ly.x_ps + (int64_t)S * P;
    ly.x_qsc = ly.x_qs + (int64_t)S * P;
    ly.x_se = ly.x_qsc + (int64_t)S * P;
    ly.x_sc = ly.x_se + (int64_t)S * P;
    ly.x_sd = ly.x_sc + (int64_t)S * P;
    ly.x_u = ly.x_sd + (int64_t)S * P;
    ly.n = ly.x_u + (int64_t)D * P;
    const int64_t rk = ly.rect, T1 = T - 1;
    const int64_t rows[B_END] = {R * P, L * P, L * P, L * P, L * P, L * P, rk * L * P, N * P, N * P, L * P, L * P,
                                 rk * N * P, (int64_t)G * T1, (int64_t)S * P, (int64_t)S * P, (int64_t)S * P,
                                 (int64_t)S * P, (int64_t)ly.comp * S * P, (int64_t)D * T1, (int64_t)D};
    ly.jbal_rep = (1 + rk) * N + G + 2LL * L + S + D;
    const int64_t angj = (2 + 2 * rk) * L * P;  // polar (va_f, va_t); rectangular (vr_f, vr_t, vi_f, vi_t)
    // state of charge: 3 entries in period 0 (se, sc, sd), 4 after (se_{t-1} too)
    const int64_t socj = (int64_t)S * (3 + 4 * (P - 1));
    const int64_t ents[B_END] = {R * P, 5LL * L * P, 5LL * L * P, 5LL * L * P, 5LL * L * P, angj, rk * angj,
                                 ly.jbal_rep * P, ly.jbal_rep * P, 2LL * L * P, 2LL * L * P, rk * 2 * N * P,
                                 2LL * G * T1, socj, 5LL * S * P, 4LL * S * P, 2LL * S * P, 2LL * ly.comp * S * P,
                                 2LL * D * T1, (int64_t)D};
    ly.c_blk[0] = ly.j_blk[0] = 0;
    for (int b = 0; b < B_END; b++) {
        ly.c_blk[b + 1] = ly.c_blk[b] + rows[b];
        ly.j_blk[b + 1] = ly.j_blk[b] + ents[b];
    }
    ly.hva_rep = hm.hva_off[N];
    ly.hvm_rep = hm.hvm_off[N];
    ly.h_va = 0;
    ly.h_vm = ly.hva_rep * P;
    ly.h_pg = ly.h_vm + ly.hvm_rep * P;
    ly.h_p = ly.h_pg + (int64_t)G * ly.npg;
    ly.h_q = ly.h_p + 2LL * L * P;
    ly.h_ps = ly.h_q + 2LL * L * P;
    ly.h_qs = ly.h_ps + 2LL * S * P;
    ly.h_sd = ly.h_qs + 2LL * S * P;
    ly.nnzh = ly.h_sd + (int64_t)ly.comp * S * P;
    if (ly.nnzh >= std::numeric_limits<int32_t>::max())
        return fail(err, OPF_E_CASE, "model too large for int32 indices");
    // the kernels address every per-instance array with 32-bit byte offsets:
    // x, c, J, H and the half-edge records (12 doubles per branch and
    // replica) must each stay below 4 GiB
    const int64_t kMaxElems = (int64_t(1) << 32) / 8;
    if (ly.n >= kMaxElems || ly.m() >= kMaxElems || ly.nnzj() >= kMaxElems || ly.nnzh >= kMaxElems ||
        12LL * L * P >= kMaxElems)
        return fail(err, OPF_E_CASE, "model too large: an array of one instance exceeds 4 GiB");
    build_slots(hm);
    return OPF_OK;
}

void build_slots(HostModel& hm) {
    const int32_t N = hm.ly.N, L = hm.ly.L;
    const bool rect = hm.ly.rect != 0;
    hm.slots.clear();
    hm.slots_c.clear();
    hm.big_bus.clear();
    int32_t lane = 0;
    auto push = [&](int32_t kind, int32_t ref, int32_t bus, int32_t other, int32_t jpos, int32_t h0, int32_t h1,
                    int32_t h2, uint32_t ckind, int32_t cidx) {
        const int32_t f[8] = {kind, ref, bus, other, jpos, h0, h1, h2};
        hm.slots.insert(hm.slots.end(), f, f + 8);
        hm.slots_c.push_back((int32_t)ckind);
        hm.slots_c.push_back(cidx);
        lane = (lane + 1) % kWaveLanes;
    };
    auto pad_wave = [&]() {
        while (lane != 0) push(SK_IDLE, -1, -1, -1, -1, -1, -1, -1, SK_IDLE, 0);
    };
    // compact kind word (SlotCompact); every field below is < 64 because a
    // segment fits one wave
    auto ck = [](uint32_t low, uint32_t len1, uint32_t head_lane, uint32_t joff, uint32_t grp) {
        return low | (len1 << 8) | (head_lane << 14) | (joff << 20) | (grp << 26);
    };
    auto group_len = [&](int32_t i, int32_t q) {
        const int32_t grp = hm.he_grp[q];
        int32_t u = q;
        while (u > hm.adj_ptr[i] && hm.he_grp[u - 1] == grp) u--;
        int32_t n = 0;
        for (; u < hm.adj_ptr[i + 1] && hm.he_grp[u] == grp; u++) n++;
        return n;
    };
    for (int32_t i = 0; i < N; i++) {
        const int32_t e0 = hm.adj_ptr[i], e1 = hm.adj_ptr[i + 1], deg = e1 - e0;
        const int32_t g0 = hm.gen_ptr[i], ng = hm.gen_ptr[i + 1] - g0;
        const int32_t s0 = hm.st_ptr[i], ns = hm.st_ptr[i + 1] - s0;
        const int32_t d0 = hm.dv_ptr[i], nd = hm.dv_ptr[i + 1] - d0;
        const int32_t seg = 1 + deg + ng + ns + nd;
        if (seg > kWaveLanes) {
            hm.big_bus.push_back(i);
            continue;
        }
        if (lane + seg > kWaveLanes) pad_wave();
        const int32_t nlo = hm.nlo[i], ndst = hm.ndist[i];
        const int32_t hva = hm.hva_off[i], hvm = hm.hvm_off[i], jrow = hm.jbal_off[i];
        const uint32_t head_lane = (uint32_t)lane;
        const int32_t nbv = rect ? 2 : 1;  // leading bus entries of the balance rows
        if (rect)  // (vr_i, vr_i), no (vi_i, vr_i), (vi_i, vi_i)
            push(SK_HEAD | (seg << 8), -1, i, -1, jrow, hva + nlo, -1, hvm + ndst + nlo,
                 ck(SK_HEAD | (deg == 0 ? 64u : 0u), seg - 1, head_lane, 0, 0), i);
        else
            push(SK_HEAD | (seg << 8), -1, i, -1, jrow, deg > 0 ? hva + nlo : -1, deg > 0 ? hvm + nlo : -1,
                 deg > 0 ? hvm + ndst + 1 + nlo : hvm, ck(SK_HEAD | (deg == 0 ? 64u : 0u), seg - 1, head_lane, 0, 0),
                 i);
        for (int32_t q = e0; q < e1; q++) {
            const int32_t code = hm.he[q], l = code >> 1, from = code & 1;
            const int32_t k = from ? hm.t_bus[l] : hm.f_bus[l];
            const int32_t grp = hm.he_grp[q];
            const bool leader = (q == e0) || hm.he_grp[q - 1] != grp;
            const int32_t glen = group_len(i, q);
            // rank of this half-edge's arc among the arcs at bus i (ascending arc index)
            const int32_t arc = from ? l : L + l;
            const auto ab = hm.arc_list.begin() + hm.arc_ptr[i], ae = hm.arc_list.begin() + hm.arc_ptr[i + 1];
            const int32_t arank = (int32_t)(std::lower_bound(ab, ae, arc) - ab);
            const int32_t kind = SK_EDGE | (from << 2) | ((leader ? 1 : 0) << 3) | ((glen > 1 ? 1 : 0) << 4) |
                                 ((leader ? glen : 0) << 8);
            const uint32_t clow = SK_EDGE | (from << 2) | ((leader ? 1u : 0u) << 3) | ((k < i ? 1u : 0u) << 4) |
                                  ((k > i ? 1u : 0u) << 5);
            if (rect)  // (vr_i, vr_k) for k < i, (vi_i, vr_k), (vi_i, vi_k) for k < i
                push(kind, l, i, k, jrow + nbv + ng + arank, leader && k < i ? hva + grp : -1,
                     leader ? hvm + grp : -1, leader && k < i ? hvm + ndst + grp : -1,
                     ck(clow, leader ? glen - 1 : 0, head_lane, 1 + ng + arank, grp), l);
            else
                push(kind, l, i, k, jrow + 1 + ng + arank, leader && k < i ? hva + grp : -1,
                     leader ? hvm + grp + (k > i ? 1 : 0) : -1, leader && k < i ? hvm + ndst + 1 + grp : -1,
                     ck(clow, leader ? glen - 1 : 0, head_lane, 1 + ng + arank, grp), l);
        }
        for (int32_t q = 0; q < ng; q++)
            push(SK_GEN, hm.gen_list[g0 + q], i, -1, jrow + nbv + q, -1, -1, -1, ck(SK_GEN, 0, head_lane, 1 + q, 0),
                 hm.gen_list[g0 + q]);
        // storage units (bit 2) and devices (bit 4): their balance entries
        // follow the arcs'; `other` is the head's lane (they read its vm)
        for (int32_t q = 0; q < ns; q++)
            push(SK_GEN | 4, hm.st_list[s0 + q], i, (int32_t)head_lane, jrow + nbv + ng + deg + q, -1, -1, -1,
                 ck(SK_GEN | 4, 0, head_lane, 1 + ng + deg + q, 0), hm.st_list[s0 + q]);
        for (int32_t q = 0; q < nd; q++)
            push(SK_GEN | 16, hm.dv_list[d0 + q], i, (int32_t)head_lane, jrow + nbv + ng + deg + ns + q, -1, -1, -1,
                 ck(SK_GEN | 16, 0, head_lane, 1 + ng + deg + ns + q, 0), hm.dv_list[d0 + q]);
    }
    pad_wave();
    hm.nwaves = (int32_t)(hm.slots.size() / (8 * kWaveLanes));
    const size_t nslot = (size_t)hm.nwaves * kWaveLanes;
    hm.slot_coef.assign(nslot * 8, 0.0);
    for (size_t q = 0; q < nslot; q++) {
        if ((hm.slots[8 * q] & 3) != SK_EDGE) continue;
        const int32_t l = hm.slots[8 * q + 1];
        for (int k = 0; k < 8; k++) hm.slot_coef[8 * q + k] = hm.coef[(size_t)k * L + l];
    }
}

void fill_pattern(const HostModel& hm, int32_t* jr, int32_t* jc, int32_t* hr, int32_t* hc) {
    const Layout& ly = hm.ly;
    const int32_t N = ly.N, L = ly.L, G = ly.G, R = ly.R, P = ly.nrep;
    auto va = [&](int32_t i, int32_t r) { return (int32_t)(ly.x_va + i + (int64_t)N * r); };
    auto vm = [&](int32_t i, int32_t r) { return (int32_t)(ly.x_vm + i + (int64_t)N * r); };
    auto pg = [&](int32_t k, int32_t r) { return (int32_t)(ly.x_pg + k + (int64_t)G * (ly.npg > 1 ? r : 0)); };
    auto qg = [&](int32_t k, int32_t r) { return (int32_t)(ly.x_qg + k + (int64_t)G * r); };
    auto pa = [&](int32_t a, int32_t r) { return (int32_t)(ly.x_p + a + 2LL * L * r); };
    auto qa = [&](int32_t a, int32_t r) { return (int32_t)(ly.x_q + a + 2LL * L * r); };
    const int32_t S = ly.S, D = ly.D;
    auto sv = [&](int64_t base, int32_t u, int32_t r) { return (int32_t)(base + u + (int64_t)S * r); };
    auto uv = [&](int32_t d, int32_t r) { return (int32_t)(ly.x_u + d + (int64_t)D * r); };

    if (jr || jc) {
        int64_t e = 0;
        int32_t row = 0;
        auto put = [&](int32_t col) {
            if (jr) jr[e] = row;
            if (jc) jc[e] = col;
            e++;
        };
        // the rectangular form reads va, vm as vr, vi (same block positions)
        const bool rect = ly.rect != 0;
        for (int32_t r = 0; r < P; r++)
            for (int32_t j = 0; j < R; j++, row++) put(rect ? vm(hm.ref_bus[j], r) : va(hm.ref_bus[j], r));
        for (int b = B_PFR; b <= B_QTO; b++) {
            const bool fr = (b == B_PFR || b == B_QFR), isp = (b == B_PFR || b == B_PTO);
            for (int32_t r = 0; r < P; r++)
                for (int32_t l = 0; l < L; l++, row++) {
                    const int32_t lo = std::min(hm.f_bus[l], hm.t_bus[l]), hi = std::max(hm.f_bus[l], hm.t_bus[l]);
                    const int32_t arc = fr ? l : L + l;
                    put(va(lo, r)); put(va(hi, r)); put(vm(lo, r)); put(vm(hi, r));
                    put(isp ? pa(arc, r) : qa(arc, r));
                }
        }
        for (int blk = 0; blk < (rect ? 2 : 1); blk++)  // angle rows (rectangular: two blocks)
            for (int32_t r = 0; r < P; r++)
                for (int32_t l = 0; l < L; l++, row++) {
                    const int32_t lo = std::min(hm.f_bus[l], hm.t_bus[l]), hi = std::max(hm.f_bus[l], hm.t_bus[l]);
                    put(va(lo, r));
                    put(va(hi, r));
                    if (rect) {
                        put(vm(lo, r));
                        put(vm(hi, r));
                    }
                }
        for (int isp = 1; isp >= 0; isp--)
            for (int32_t r = 0; r < P; r++)
                for (int32_t i = 0; i < N; i++, row++) {
                    if (rect) put(va(i, r));
                    put(vm(i, r));
                    for (int32_t q = hm.gen_ptr[i]; q < hm.gen_ptr[i + 1]; q++)
                        put(isp ? pg(hm.gen_list[q], r) : qg(hm.gen_list[q], r));
                    for (int32_t q = hm.arc_ptr[i]; q < hm.arc_ptr[i + 1]; q++)
                        put(isp ? pa(hm.arc_list[q], r) : qa(hm.arc_list[q], r));
                    for (int32_t q = hm.st_ptr[i]; q < hm.st_ptr[i + 1]; q++)
                        put(sv(isp ? ly.x_ps : ly.x_qs, hm.st_list[q], r));
                    for (int32_t q = hm.dv_ptr[i]; q < hm.dv_ptr[i + 1]; q++) put(uv(hm.dv_list[q], r));
                }
        for (int side = 0; side < 2; side++)
            for (int32_t r = 0; r < P; r++)
                for (int32_t l = 0; l < L; l++, row++) {
                    const int32_t arc = side == 0 ? l : L + l;
                    put(pa(arc, r));
                    put(qa(arc, r));
                }
        if (rect)  // voltage-magnitude rows
            for (int32_t r = 0; r < P; r++)
                for (int32_t i = 0; i < N; i++, row++) {
                    put(va(i, r));
                    put(vm(i, r));
                }
        for (int32_t t = 1; t < ly.T; t++)
            for (int32_t k = 0; k < G; k++, row++) {
                put(pg(k, t - 1));
                put(pg(k, t));
            }
        // storage rows, columns ascending: soc [se_{t-1}], se, sc, sd; loss_p
        // vm, ps, qs, sc, sd; loss_q vm, ps, qs, qsc; thermal ps, qs; comp sc, sd
        for (int32_t r = 0; r < P; r++)
            for (int32_t u = 0; u < S; u++, row++) {
                if (r >= 1) put(sv(ly.x_se, u, r - 1));
                put(sv(ly.x_se, u, r));
                put(sv(ly.x_sc, u, r));
                put(sv(ly.x_sd, u, r));
            }
        for (int32_t r = 0; r < P; r++)
            for (int32_t u = 0; u < S; u++, row++) {
                put(vm(hm.stor_bus[u], r));
                put(sv(ly.x_ps, u, r));
                put(sv(ly.x_qs, u, r));
                put(sv(ly.x_sc, u, r));
                put(sv(ly.x_sd, u, r));
            }
        for (int32_t r = 0; r < P; r++)
            for (int32_t u = 0; u < S; u++, row++) {
                put(vm(hm.stor_bus[u], r));
                put(sv(ly.x_ps, u, r));
                put(sv(ly.x_qs, u, r));
                put(sv(ly.x_qsc, u, r));
            }
        for (int32_t r = 0; r < P; r++)
            for (int32_t u = 0; u < S; u++, row++) {
                put(sv(ly.x_ps, u, r));
                put(sv(ly.x_qs, u, r));
            }
        for (int32_t r = 0; r < P && ly.comp; r++)
            for (int32_t u = 0; u < S; u++, row++) {
                put(sv(ly.x_sc, u, r));
                put(sv(ly.x_sd, u, r));
            }
        // device rows: ramp u_{t-1}, u_t; init u_0
        for (int32_t t = 1; t < ly.T; t++)
            for (int32_t d = 0; d < D; d++, row++) {
                put(uv(d, t - 1));
                put(uv(d, t));
            }
        for (int32_t d = 0; d < D; d++, row++) put(uv(d, 0));
    }

    if (hr || hc) {
        int64_t e = 0;
        auto put = [&](int32_t row, int32_t col) {
            if (hr) hr[e] = row;
            if (hc) hc[e] = col;
            e++;
        };
        auto nbr = [&](int32_t code) {
            const int32_t l = code >> 1;
            return (code & 1) ? hm.t_bus[l] : hm.f_bus[l];
        };
        // distinct neighbours of bus i, ascending (one per group)
        auto distinct = [&](int32_t i, std::vector<int32_t>& out) {
            out.clear();
            for (int32_t q = hm.adj_ptr[i]; q < hm.adj_ptr[i + 1]; q++) {
                const int32_t k = nbr(hm.he[q]);
                if (out.empty() || out.back() != k) out.push_back(k);
            }
        };
        std::vector<int32_t> nb;
        if (ly.rect) {
            // vr row i: (vr_i, vr_k) for k < i, diagonal; vi row i: (vi_i, vr_k)
            // for every distinct neighbour, (vi_i, vi_k) for k < i, diagonal
            for (int32_t r = 0; r < P; r++)
                for (int32_t i = 0; i < N; i++) {
                    distinct(i, nb);
                    for (int32_t k : nb)
                        if (k < i) put(va(i, r), va(k, r));
                    put(va(i, r), va(i, r));
                }
            for (int32_t r = 0; r < P; r++)
                for (int32_t i = 0; i < N; i++) {
                    distinct(i, nb);
                    for (int32_t k : nb) put(vm(i, r), va(k, r));
                    for (int32_t k : nb)
                        if (k < i) put(vm(i, r), vm(k, r));
                    put(vm(i, r), vm(i, r));
                }
        }
        for (int32_t r = 0; r < P && !ly.rect; r++)
            for (int32_t i = 0; i < N; i++) {
                distinct(i, nb);
                if (nb.empty()) continue;
                for (int32_t k : nb)
                    if (k < i) put(va(i, r), va(k, r));
                put(va(i, r), va(i, r));
            }
        for (int32_t r = 0; r < P && !ly.rect; r++)
            for (int32_t i = 0; i < N; i++) {
                distinct(i, nb);
                if (!nb.empty()) {
                    for (int32_t k : nb)
                        if (k < i) put(vm(i, r), va(k, r));
                    put(vm(i, r), va(i, r));
                    for (int32_t k : nb)
                        if (k > i) put(vm(i, r), va(k, r));
                    for (int32_t k : nb)
                        if (k < i) put(vm(i, r), vm(k, r));
                }
                put(vm(i, r), vm(i, r));
            }
        for (int32_t r = 0; r < ly.npg; r++)
            for (int32_t k = 0; k < G; k++) put(pg(k, r), pg(k, r));
        for (int32_t r = 0; r < P; r++)
            for (int32_t a = 0; a < 2 * L; a++) put(pa(a, r), pa(a, r));
        for (int32_t r = 0; r < P; r++)
            for (int32_t a = 0; a < 2 * L; a++) put(qa(a, r), qa(a, r));
        // storage rows: (ps, vm), (ps, ps); (qs, vm), (qs, qs); (sd, sc)
        for (int32_t r = 0; r < P; r++)
            for (int32_t u = 0; u < S; u++) {
                put(sv(ly.x_ps, u, r), vm(hm.stor_bus[u], r));
                put(sv(ly.x_ps, u, r), sv(ly.x_ps, u, r));
            }
        for (int32_t r = 0; r < P; r++)
            for (int32_t u = 0; u < S; u++) {
                put(sv(ly.x_qs, u, r), vm(hm.stor_bus[u], r));
                put(sv(ly.x_qs, u, r), sv(ly.x_qs, u, r));
            }
        for (int32_t r = 0; r < P && ly.comp; r++)
            for (int32_t u = 0; u < S; u++) put(sv(ly.x_sd, u, r), sv(ly.x_sc, u, r));
    }
}

void fill_bounds(const opf_case* cs, const opf_opts* opts, const HostModel& hm, double* lvar, double* uvar,
                 double* lcon, double* ucon, double* x0) {
    const Layout& ly = hm.ly;
    const int32_t N = ly.N, L = ly.L, G = ly.G, P = ly.nrep;
    const double inf = std::numeric_limits<double>::infinity();
    if (lvar || uvar || x0) {
        for (int64_t j = 0; j < ly.n; j++) {
            if (lvar) lvar[j] = -inf;
            if (uvar) uvar[j] = inf;
            if (x0) x0[j] = 0.0;
        }
        for (int32_t r = 0; r < P; r++) {
            for (int32_t i = 0; i < N; i++) {
                const int64_t c = ly.x_vm + i + (int64_t)N * r;
                if (ly.rect) {  // vr, vi in [-vmax, vmax]; start vr = 1, vi = 0
                    const int64_t cr = ly.x_va + i + (int64_t)N * r;
                    if (lvar) lvar[cr] = lvar[c] = -cs->vmax[i];
                    if (uvar) uvar[cr] = uvar[c] = cs->vmax[i];
                    if (x0) x0[cr] = 1.0;
                    continue;
                }
                if (lvar) lvar[c] = cs->vmin[i];
                if (uvar) uvar[c] = cs->vmax[i];
                if (x0) x0[c] = 1.0;
            }
            for (int32_t k = 0; k < G; k++) {
                const int64_t c = ly.x_qg + k + (int64_t)G * r;
                if (lvar) lvar[c] = cs->qmin[k];
                if (uvar) uvar[c] = cs->qmax[k];
            }
            for (int32_t a = 0; a < 2 * L; a++) {
                const double rate = cs->rate_a[a < L ? a : a - L];
                const int64_t cp = ly.x_p + a + 2LL * L * r, cq = ly.x_q + a + 2LL * L * r;
                if (lvar) { lvar[cp] = -rate; lvar[cq] = -rate; }
                if (uvar) { uvar[cp] = rate; uvar[cq] = rate; }
            }
        }
        for (int32_t r = 0; r < ly.npg; r++)
            for (int32_t k = 0; k < G; k++) {
                const int64_t c = ly.x_pg + k + (int64_t)G * r;
                if (lvar) lvar[c] = cs->pmin[k];
                if (uvar) uvar[c] = cs->pmax[k];
            }
        const int32_t S = ly.S, D = ly.D;
        for (int32_t r = 0; r < P; r++) {
            for (int32_t u = 0; u < S; u++) {
                const opf_storage* st = opts->storage;
                const int64_t o = u + (int64_t)S * r;
                const double lo[6] = {-st->rating[u], st->qmin[u], -st->rating[u], 0.0, 0.0, 0.0};
                const double hi[6] = {st->rating[u], st->qmax[u], st->rating[u], st->emax[u], st->chmax[u],
                                      st->dismax[u]};
                const int64_t base[6] = {ly.x_ps, ly.x_qs, ly.x_qsc, ly.x_se, ly.x_sc, ly.x_sd};
                for (int k = 0; k < 6; k++) {
                    if (lvar) lvar[base[k] + o] = lo[k];
                    if (uvar) uvar[base[k] + o] = hi[k];
                }
            }
            for (int32_t d = 0; d < D; d++) {
                const int64_t c = ly.x_u + d + (int64_t)D * r;
                if (lvar) lvar[c] = opts->devices->lo[d];
                if (uvar) uvar[c] = opts->devices->hi[d];
            }
        }
    }
    if (lcon || ucon) {
        const int64_t m = ly.m();
        for (int64_t j = 0; j < m; j++) {
            if (lcon) lcon[j] = 0.0;
            if (ucon) ucon[j] = 0.0;
        }
        for (int32_t r = 0; r < P; r++)
            for (int32_t l = 0; l < L; l++) {
                const int64_t row = ly.c_blk[B_ANG] + l + (int64_t)L * r;
                const bool out = hm.outage[r] == l;
                if (ly.rect) {  // SI - tan(angmax) CR <= 0, SI - tan(angmin) CR >= 0
                    const int64_t rlo = ly.c_blk[B_ANGL] + l + (int64_t)L * r;
                    if (lcon) lcon[row] = -inf;
                    if (ucon) ucon[row] = out ? inf : 0.0;
                    if (lcon) lcon[rlo] = out ? -inf : 0.0;
                    if (ucon) ucon[rlo] = inf;
                    continue;
                }
                if (lcon) lcon[row] = out ? -inf : cs->angmin[l];
                if (ucon) ucon[row] = out ? inf : cs->angmax[l];
            }
        for (int64_t row = ly.c_blk[B_THF]; row < ly.c_blk[B_VMAG]; row++)
            if (lcon) lcon[row] = -inf;
        // storage thermal and complementarity rows: (-inf, 0]; device rows
        for (int64_t row = ly.c_blk[B_STH]; row < ly.c_blk[B_DRAMP]; row++)
            if (lcon) lcon[row] = -inf;
        for (int32_t t = 1; t < ly.T; t++)
            for (int32_t d = 0; d < ly.D; d++) {
                const int64_t row = ly.c_blk[B_DRAMP] + d + (int64_t)ly.D * (t - 1);
                if (lcon) lcon[row] = -opts->devices->ramp[d];
                if (ucon) ucon[row] = opts->devices->ramp[d];
            }
        for (int32_t d = 0; d < ly.D; d++) {
            const int64_t row = ly.c_blk[B_DINIT] + d;
            if (lcon) lcon[row] = opts->devices->init_lo[d];
            if (ucon) ucon[row] = opts->devices->init_hi[d];
        }
        for (int32_t r = 0; r < P && ly.rect; r++)
            for (int32_t i = 0; i < N; i++) {
                const int64_t row = ly.c_blk[B_VMAG] + i + (int64_t)N * r;
                if (lcon) lcon[row] = cs->vmin[i] * cs->vmin[i];
                if (ucon) ucon[row] = cs->vmax[i] * cs->vmax[i];
            }
        const double ratio = opts ? opts->ramp_ratio : 0.0;
        for (int32_t t = 1; t < ly.T; t++)
            for (int32_t k = 0; k < G; k++) {
                const int64_t row = ly.c_blk[B_RAMP] + k + (int64_t)G * (t - 1);
                if (lcon) lcon[row] = -ratio * cs->pmax[k];
                if (ucon) ucon[row] = ratio * cs->pmax[k];
            }
    }
}

}  // namespace opf
