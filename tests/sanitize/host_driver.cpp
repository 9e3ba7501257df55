// Sanitizer driver for the host model code (validation, branch terms,
// adjacency, wave packing, patterns, bounds): built with g++ and
// -fsanitize=address,undefined by tests/test_sanitize.py and run over
// static, multi-period, contingency, rectangular, storage and device
// models, a bus wider than a wave, and malformed inputs.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "host_model.h"

extern "C" {
#include "cases.h"
}

namespace {

int run(const san_net& n, const opf_opts* o, bool expect_ok) {
    opf_case cs{};
    cs.n_bus = n.N; cs.n_branch = n.L; cs.n_gen = n.G; cs.n_ref = 1;
    cs.pd = n.pd; cs.qd = n.qd; cs.gs = n.gs; cs.bs = n.bs; cs.vmin = n.vmin; cs.vmax = n.vmax;
    cs.ref_bus = n.ref_bus; cs.f_bus = n.f_bus; cs.t_bus = n.t_bus;
    cs.r = n.r; cs.x = n.x; cs.b = n.b; cs.tap = n.tap; cs.shift = n.shift; cs.rate_a = n.rate;
    cs.angmin = n.angmin; cs.angmax = n.angmax; cs.gen_bus = n.gen_bus;
    cs.pmin = n.pmin; cs.pmax = n.pmax; cs.qmin = n.qmin; cs.qmax = n.qmax; cs.c2 = n.c2; cs.c1 = n.c1; cs.c0 = n.c0;
    opf::HostModel hm;
    std::string err;
    const int rc = opf::build_host_model(&cs, o, hm, err);
    if ((rc == OPF_OK) != expect_ok) {
        std::fprintf(stderr, "unexpected status %d (%s)\n", rc, err.c_str());
        return 1;
    }
    if (rc != OPF_OK) return 0;
    const opf::Layout& ly = hm.ly;
    std::vector<int32_t> jr(ly.nnzj()), jc(ly.nnzj()), hr(ly.nnzh), hc(ly.nnzh);
    opf::fill_pattern(hm, jr.data(), jc.data(), hr.data(), hc.data());
    std::vector<double> lv(ly.n), uv(ly.n), lc(ly.m()), uc(ly.m()), x0(ly.n);
    opf::fill_bounds(&cs, o, hm, lv.data(), uv.data(), lc.data(), uc.data(), x0.data());
    for (int64_t e = 1; e < ly.nnzj(); e++)
        if (jr[e] < jr[e - 1] || (jr[e] == jr[e - 1] && jc[e] <= jc[e - 1])) {
            std::fprintf(stderr, "Jacobian pattern not sorted at %lld\n", (long long)e);
            return 1;
        }
    for (int64_t e = 0; e < ly.nnzh; e++)
        if (hr[e] < hc[e] || hr[e] >= ly.n) {
            std::fprintf(stderr, "Hessian entry %lld outside the lower triangle\n", (long long)e);
            return 1;
        }
    return 0;
}

}  // namespace

int main() {
    int bad = 0;
    san_net a, b;
    san_make(&a, 60, 25, 12, 0, 0, 0, 1);
    san_make(&b, 200, 40, 30, 8, 6, 70, 2);  // bus 0 joins 70 more branches: a wide bus
    std::vector<double> pdt(4 * 200), qdt(4 * 200);
    for (int k = 0; k < 800; k++) { pdt[k] = b.pd[k % 200]; qdt[k] = b.qd[k % 200]; }
    int32_t out[3] = {3, 7, 11};
    opf_storage st{};
    st.n = b.S; st.bus = b.stor_bus;
    st.emax = b.st[0]; st.chmax = b.st[1]; st.dismax = b.st[2]; st.rating = b.st[3]; st.qmin = b.st[4];
    st.qmax = b.st[5]; st.eta_c = b.st[6]; st.eta_d = b.st[7]; st.r = b.st[8]; st.x = b.st[9];
    st.ploss = b.st[10]; st.qloss = b.st[11]; st.e0 = b.st[12]; st.dt = 0.5; st.comp = 1;
    opf_devices dv{};
    dv.n = b.D; dv.bus = b.dev_bus; dv.cp = b.dv[0]; dv.cq = b.dv[1]; dv.cost = b.dv[2]; dv.lo = b.dv[3];
    dv.hi = b.dv[4]; dv.ramp = b.dv[5]; dv.init_lo = b.dv[6]; dv.init_hi = b.dv[7];

    opf_opts mp{}; mp.n_periods = 4; mp.pd_t = pdt.data(); mp.qd_t = qdt.data(); mp.ramp_ratio = 0.2;
    opf_opts sc{}; sc.n_periods = 1; sc.n_cont = 3; sc.outaged_branch = out;
    opf_opts rect{}; rect.n_periods = 2; rect.ramp_ratio = 0.2; rect.form = OPF_FORM_RECT; rect.devices = &dv;
    opf_opts ext = mp; ext.storage = &st; ext.devices = &dv;
    opf_opts rect_sc = sc; rect_sc.form = OPF_FORM_RECT;
    bad |= run(a, nullptr, true);
    bad |= run(a, &sc, true);
    bad |= run(b, &mp, true);
    bad |= run(b, &ext, true);
    bad |= run(b, &rect, true);
    bad |= run(b, &rect_sc, true);
    // malformed: storage with contingency copies, rectangular storage,
    // a bus out of range, a zero-impedance branch
    opf_opts bad1 = sc; bad1.storage = &st;
    opf_opts bad2 = ext; bad2.form = OPF_FORM_RECT;
    bad |= run(b, &bad1, false);
    bad |= run(b, &bad2, false);
    b.f_bus[5] = 999;
    bad |= run(b, &mp, false);
    b.f_bus[5] = 0;
    b.r[6] = 0.0; b.x[6] = 0.0;
    bad |= run(b, &mp, false);
    san_free(&a);
    san_free(&b);
    std::printf(bad ? "host driver: FAILED\n" : "host driver: ok\n");
    return bad;
}
