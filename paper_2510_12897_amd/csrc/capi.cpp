// C-ABI of libopf (declared in include/opf.h): models and callbacks.
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>
#include <tuple>

#include "internal.h"

namespace opf_internal {

namespace {
thread_local std::string g_err;
std::mutex g_alloc_mu;
void* (*g_alloc)(size_t, void*) = nullptr;
void (*g_release)(void*, void*) = nullptr;
void* g_alloc_ctx = nullptr;
}  // namespace

const std::string& last_error() { return g_err; }

void set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = alloc;
    g_release = release;
    g_alloc_ctx = ctx;
}

int set_err(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_err(hipError_t e, const char* what) {
    return set_err(OPF_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

Allocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return Allocator{g_alloc, g_release, g_alloc_ctx};
}

void* dev_alloc(const Allocator& a, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (a.alloc) return a.alloc(bytes, a.ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void dev_free(const Allocator& a, void* p) {
    if (!p) return;
    if (a.release)
        a.release(p, a.ctx);
    else
        (void)hipFree(p);
}

ModelOffsets pack_model(Packer& pk, const opf::HostModel& hm) {
    ModelOffsets o{};
    o.f_bus = pk.add(hm.f_bus);
    o.t_bus = pk.add(hm.t_bus);
    o.coef = pk.add(hm.coef);
    o.rate2 = pk.add(hm.rate2);
    o.slots = pk.add(hm.slots);
    o.slot_coef = pk.add(hm.slot_coef);
    o.big_bus = pk.add(hm.big_bus);
    o.adj_ptr = pk.add(hm.adj_ptr);
    o.he = pk.add(hm.he);
    o.he_grp = pk.add(hm.he_grp);
    o.nlo = pk.add(hm.nlo);
    o.ndist = pk.add(hm.ndist);
    o.hva_off = pk.add(hm.hva_off);
    o.hvm_off = pk.add(hm.hvm_off);
    o.jbal_off = pk.add(hm.jbal_off);
    o.gen_ptr = pk.add(hm.gen_ptr);
    o.gen_list = pk.add(hm.gen_list);
    o.gs = pk.add(hm.gs);
    o.bs = pk.add(hm.bs);
    o.pd = pk.add(hm.pd);
    o.qd = pk.add(hm.qd);
    o.c2 = pk.add(hm.c2);
    o.c1 = pk.add(hm.c1);
    o.c0 = pk.add(hm.c0);
    o.gen_bus = pk.add(hm.gen_bus);
    o.ref_bus = pk.add(hm.ref_bus);
    o.ref_ptr = pk.add(hm.ref_ptr);
    o.ref_list = pk.add(hm.ref_list);
    o.outage = pk.add(hm.outage);
    o.slots_c = pk.add(hm.slots_c);
    o.tan_lim = pk.add(hm.tan_lim);
    o.stor_bus = pk.add(hm.stor_bus);
    o.stor_par = pk.add(hm.stor_par);
    o.dev_bus = pk.add(hm.dev_bus);
    o.dev_par = pk.add(hm.dev_par);
    o.st_ptr = pk.add(hm.st_ptr);
    o.st_list = pk.add(hm.st_list);
    o.dv_ptr = pk.add(hm.dv_ptr);
    o.dv_list = pk.add(hm.dv_list);
    return o;
}

namespace {
std::atomic<int64_t> g_single_launch_limit{4096};
int64_t single_launch_limit() { return g_single_launch_limit.load(); }
int32_t gen_chunks(const opf::HostModel& hm) {
    return (std::max(hm.ly.G, hm.ly.R) + opf::kBlock - 1) / opf::kBlock;
}
size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

void attach_scratch(opf::DevModel& d, char* scratch) {
    const size_t parts = round256(sizeof(double) * (size_t)opf::obj_slots(d));
    d.obj_part = reinterpret_cast<double*>(scratch);
    d.obj_ticket = reinterpret_cast<int32_t*>(scratch + parts);
    d.rec = reinterpret_cast<double*>(scratch + parts + 256);
}

opf::DevModel make_dev(const opf::HostModel& hm, char* base, const ModelOffsets& o) {
    const opf::Layout& ly = hm.ly;
    opf::DevModel d{};
    d.N = ly.N; d.L = ly.L; d.G = ly.G; d.R = ly.R; d.T = ly.T;
    d.nrep = ly.nrep; d.npg = ly.npg; d.load_stride = hm.load_stride;
    d.nwaves = hm.nwaves;
    d.nbig = (int32_t)hm.big_bus.size();
    d.big_cap = 0;
    for (int32_t b : hm.big_bus) d.big_cap = std::max(d.big_cap, hm.adj_ptr[b + 1] - hm.adj_ptr[b]);
    d.nbchunks = (ly.L + opf::kBlock - 1) / opf::kBlock;
    d.ngchunks = gen_chunks(hm);
    // one launch per callback set when the whole set is a few waves per
    // compute unit (the launch is latency-bound)
    d.S = ly.S;
    d.D = ly.D;
    d.nschunks = (ly.S + opf::kBlock - 1) / opf::kBlock;
    d.ndchunks = (ly.D + opf::kBlock - 1) / opf::kBlock;
    d.comp = ly.comp;
    const int64_t waves = (int64_t)ly.nrep * (d.nbchunks + d.nwaves + d.nbig + d.ngchunks + d.nschunks + d.ndchunks);
    const int64_t limit = single_launch_limit();
    d.single = (limit > 0 && waves <= limit) ? 1 : 0;
    d.x_va = ly.x_va; d.x_vm = ly.x_vm; d.x_pg = ly.x_pg; d.x_qg = ly.x_qg; d.x_p = ly.x_p; d.x_q = ly.x_q;
    using namespace opf;
    d.c_ref = ly.c_blk[B_REF]; d.c_pfr = ly.c_blk[B_PFR]; d.c_qfr = ly.c_blk[B_QFR];
    d.c_pto = ly.c_blk[B_PTO]; d.c_qto = ly.c_blk[B_QTO]; d.c_ang = ly.c_blk[B_ANG];
    d.c_balp = ly.c_blk[B_BALP]; d.c_balq = ly.c_blk[B_BALQ]; d.c_thf = ly.c_blk[B_THF];
    d.c_tht = ly.c_blk[B_THT]; d.c_ramp = ly.c_blk[B_RAMP];
    d.j_ref = ly.j_blk[B_REF]; d.j_pfr = ly.j_blk[B_PFR]; d.j_qfr = ly.j_blk[B_QFR];
    d.j_pto = ly.j_blk[B_PTO]; d.j_qto = ly.j_blk[B_QTO]; d.j_ang = ly.j_blk[B_ANG];
    d.j_balp = ly.j_blk[B_BALP]; d.j_balq = ly.j_blk[B_BALQ]; d.j_thf = ly.j_blk[B_THF];
    d.j_tht = ly.j_blk[B_THT]; d.j_ramp = ly.j_blk[B_RAMP]; d.jbal_rep = ly.jbal_rep;
    d.h_va = ly.h_va; d.h_vm = ly.h_vm; d.h_pg = ly.h_pg; d.h_p = ly.h_p; d.h_q = ly.h_q;
    d.hva_rep = ly.hva_rep; d.hvm_rep = ly.hvm_rep;
#define P32(name) d.name = reinterpret_cast<const int32_t*>(base + o.name)
#define PDB(name) d.name = reinterpret_cast<const double*>(base + o.name)
    P32(f_bus); P32(t_bus); PDB(coef); PDB(rate2); P32(slots); PDB(slot_coef); P32(big_bus);
    P32(adj_ptr); P32(he); P32(he_grp); P32(nlo); P32(ndist); P32(hva_off); P32(hvm_off); P32(jbal_off);
    P32(gen_ptr); P32(gen_list); PDB(gs); PDB(bs); PDB(pd); PDB(qd);
    PDB(c2); PDB(c1); PDB(c0); P32(gen_bus); P32(ref_bus); P32(ref_ptr); P32(ref_list); P32(outage); P32(slots_c);
    PDB(tan_lim);
    P32(stor_bus); PDB(stor_par); P32(dev_bus); PDB(dev_par); P32(st_ptr); P32(st_list); P32(dv_ptr); P32(dv_list);
    d.x_ps = ly.x_ps; d.x_qs = ly.x_qs; d.x_qsc = ly.x_qsc; d.x_se = ly.x_se; d.x_sc = ly.x_sc; d.x_sd = ly.x_sd;
    d.x_u = ly.x_u;
    d.c_soc = ly.c_blk[B_SOC]; d.c_slp = ly.c_blk[B_SLP]; d.c_slq = ly.c_blk[B_SLQ]; d.c_sth = ly.c_blk[B_STH];
    d.c_scmp = ly.c_blk[B_SCMP]; d.c_dramp = ly.c_blk[B_DRAMP]; d.c_dinit = ly.c_blk[B_DINIT];
    d.j_soc = ly.j_blk[B_SOC]; d.j_slp = ly.j_blk[B_SLP]; d.j_slq = ly.j_blk[B_SLQ]; d.j_sth = ly.j_blk[B_STH];
    d.j_scmp = ly.j_blk[B_SCMP]; d.j_dramp = ly.j_blk[B_DRAMP]; d.j_dinit = ly.j_blk[B_DINIT];
    d.h_ps = ly.h_ps; d.h_qs = ly.h_qs; d.h_sd = ly.h_sd;
    d.stor_dt = hm.stor_dt;
    d.rect = ly.rect;
    d.c_angl = ly.c_blk[B_ANGL]; d.c_vmag = ly.c_blk[B_VMAG];
    d.j_angl = ly.j_blk[B_ANGL]; d.j_vmag = ly.j_blk[B_VMAG];
#undef P32
#undef PDB
    return d;
}

}  // namespace opf_internal

using namespace opf_internal;

namespace {

bool valid(const opf_model_s* m) { return valid_model(m); }

int check_model(opf_model m) {
    if (!valid(m)) return set_err(OPF_E_STATE, "invalid or destroyed model handle");
    return OPF_OK;
}

int launch_set(opf_model m, const opf::EvalOut& o, void* stream) {
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) return hip_err(dg.err, "hipSetDevice");
    hipError_t e = opf::launch_eval_set(m->dm, o, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_err(e, "callback kernel launch");
    return OPF_OK;
}

}  // namespace

// ======================================================================== API
extern "C" {

const char* opf_last_error(void) { return last_error().c_str(); }

void opf_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
    set_allocator(alloc, release, ctx);
}

int opf_set_single_launch_limit(int64_t waves) {
    if (waves < 0) return set_err(OPF_E_ARG, "the limit must be >= 0");
    g_single_launch_limit.store(waves);
    return OPF_OK;
}

int opf_case_validate(const opf_case* cs, const opf_opts* opts) {
    std::string err;
    int rc = opf::validate(cs, opts, err);
    if (rc) return set_err(rc, "%s", err.c_str());
    return OPF_OK;
}

int opf_case_dims(const opf_case* cs, const opf_opts* opts, int64_t* n, int64_t* m, int64_t* nnzj,
                  int64_t* nnzh) {
    opf::HostModel hm;
    std::string err;
    int rc;
    try {
        rc = opf::build_host_model(cs, opts, hm, err);
    } catch (const std::bad_alloc&) {
        return set_err(OPF_E_NOMEM, "host allocation failed");
    }
    if (rc) return set_err(rc, "%s", err.c_str());
    if (n) *n = hm.ly.n;
    if (m) *m = hm.ly.m();
    if (nnzj) *nnzj = hm.ly.nnzj();
    if (nnzh) *nnzh = hm.ly.nnzh;
    return OPF_OK;
}

int opf_case_structure(const opf_case* cs, const opf_opts* opts, int32_t* jrows, int32_t* jcols, int32_t* hrows,
                       int32_t* hcols) {
    opf::HostModel hm;
    std::string err;
    try {
        int rc = opf::build_host_model(cs, opts, hm, err);
        if (rc) return set_err(rc, "%s", err.c_str());
        opf::fill_pattern(hm, jrows, jcols, hrows, hcols);
    } catch (const std::bad_alloc&) {
        return set_err(OPF_E_NOMEM, "host allocation failed");
    }
    return OPF_OK;
}

int opf_case_bounds(const opf_case* cs, const opf_opts* opts, double* lvar, double* uvar, double* lcon,
                    double* ucon, double* x0) {
    opf::HostModel hm;
    std::string err;
    try {
        int rc = opf::build_host_model(cs, opts, hm, err);
        if (rc) return set_err(rc, "%s", err.c_str());
        opf::fill_bounds(cs, opts, hm, lvar, uvar, lcon, ucon, x0);
    } catch (const std::bad_alloc&) {
        return set_err(OPF_E_NOMEM, "host allocation failed");
    }
    return OPF_OK;
}

int opf_model_create(const opf_case* cs, const opf_opts* opts, int device, opf_model* out) {
    if (!out) return set_err(OPF_E_ARG, "out is NULL");
    *out = nullptr;
    opf_model_s* m = nullptr;
    try {
        m = new opf_model_s();
        std::string err;
        int rc = opf::build_host_model(cs, opts, m->hm, err);
        if (rc) {
            delete m;
            return set_err(rc, "%s", err.c_str());
        }
        m->device = device;
        m->alloc = current_allocator();
        const opf::Layout& ly = m->hm.ly;

        Packer pk;
        ModelOffsets mo = pack_model(pk, m->hm);
        opf::DevModel probe = make_dev(m->hm, nullptr, mo);
        const size_t o_scr = pk.reserve(opf::scratch_bytes(probe));  // zeroed: the ticket starts at 0
        const size_t oj_r = pk.reserve(sizeof(int32_t) * ly.nnzj());
        const size_t oj_c = pk.reserve(sizeof(int32_t) * ly.nnzj());
        const size_t oh_r = pk.reserve(sizeof(int32_t) * ly.nnzh);
        const size_t oh_c = pk.reserve(sizeof(int32_t) * ly.nnzh);
        opf::fill_pattern(m->hm, reinterpret_cast<int32_t*>(pk.at(oj_r)), reinterpret_cast<int32_t*>(pk.at(oj_c)),
                          reinterpret_cast<int32_t*>(pk.at(oh_r)), reinterpret_cast<int32_t*>(pk.at(oh_c)));
        const size_t ob_lv = pk.reserve(sizeof(double) * ly.n), ob_uv = pk.reserve(sizeof(double) * ly.n);
        const size_t ob_lc = pk.reserve(sizeof(double) * ly.m()), ob_uc = pk.reserve(sizeof(double) * ly.m());
        const size_t ob_x0 = pk.reserve(sizeof(double) * ly.n);
        const size_t o_isref = pk.add(m->hm.is_ref);
        std::vector<int32_t> he_pos(2 * (size_t)ly.L), gen_pos(ly.G);
        for (size_t h = 0; h < m->hm.he.size(); h++) {
            const int32_t code = m->hm.he[h];
            he_pos[((code & 1) ? 0 : ly.L) + (code >> 1)] = (int32_t)h;
        }
        for (size_t q = 0; q < m->hm.gen_list.size(); q++) gen_pos[m->hm.gen_list[q]] = (int32_t)q;
        const size_t o_hepos = pk.add(he_pos), o_genpos = pk.add(gen_pos);
        opf::fill_bounds(cs, opts, m->hm, reinterpret_cast<double*>(pk.at(ob_lv)),
                         reinterpret_cast<double*>(pk.at(ob_uv)), reinterpret_cast<double*>(pk.at(ob_lc)),
                         reinterpret_cast<double*>(pk.at(ob_uc)), reinterpret_cast<double*>(pk.at(ob_x0)));

        DeviceGuard dg(device);
        if (dg.err != hipSuccess) {
            delete m;
            return hip_err(dg.err, "hipSetDevice");
        }
        m->arena = dev_alloc(m->alloc, pk.buf.size());
        if (!m->arena) {
            delete m;
            return set_err(OPF_E_NOMEM, "device allocation of %zu bytes failed", pk.buf.size());
        }
        hipError_t e = hipMemcpy(m->arena, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dev_free(m->alloc, m->arena);
            delete m;
            return hip_err(e, "model upload");
        }
        char* base = static_cast<char*>(m->arena);
        m->dm = make_dev(m->hm, base, mo);
        attach_scratch(m->dm, base + o_scr);
        m->jrow = reinterpret_cast<const int32_t*>(base + oj_r);
        m->jcol = reinterpret_cast<const int32_t*>(base + oj_c);
        m->hrow = reinterpret_cast<const int32_t*>(base + oh_r);
        m->hcol = reinterpret_cast<const int32_t*>(base + oh_c);
        m->lvar = reinterpret_cast<const double*>(base + ob_lv);
        m->uvar = reinterpret_cast<const double*>(base + ob_uv);
        m->lcon = reinterpret_cast<const double*>(base + ob_lc);
        m->ucon = reinterpret_cast<const double*>(base + ob_uc);
        m->x0 = reinterpret_cast<const double*>(base + ob_x0);
        m->is_ref = reinterpret_cast<const int32_t*>(base + o_isref);
        m->he_pos = reinterpret_cast<const int32_t*>(base + o_hepos);
        m->gen_pos = reinterpret_cast<const int32_t*>(base + o_genpos);
    } catch (const std::bad_alloc&) {
        delete m;
        return set_err(OPF_E_NOMEM, "host allocation failed");
    }
    *out = m;
    return OPF_OK;
}

int opf_model_destroy(opf_model m) {
    if (!m) return OPF_OK;
    if (!valid(m)) return set_err(OPF_E_STATE, "invalid or destroyed model handle");
    {
        DeviceGuard dg(m->device);
        (void)hipDeviceSynchronize();
        dev_free(m->alloc, m->arena);
    }
    m->magic = 0;
    delete m;
    return OPF_OK;
}

int opf_model_dims(opf_model m, int64_t* n, int64_t* mm, int64_t* nnzj, int64_t* nnzh) {
    if (int rc = check_model(m)) return rc;
    const opf::Layout& ly = m->hm.ly;
    if (n) *n = ly.n;
    if (mm) *mm = ly.m();
    if (nnzj) *nnzj = ly.nnzj();
    if (nnzh) *nnzh = ly.nnzh;
    return OPF_OK;
}

int opf_model_launches(opf_model m, int32_t* launches, int64_t* items) {
    if (int rc = check_model(m)) return rc;
    const opf::DevModel& d = m->dm;
    if (launches) *launches = d.single ? 1 : 2;
    if (items)
        *items = (int64_t)d.nrep * ((int64_t)d.nbchunks + d.nwaves + d.nbig + d.ngchunks + d.nschunks + d.ndchunks);
    return OPF_OK;
}

int opf_model_blocks(opf_model m, int32_t which, int64_t* offset, int64_t* len) {
    if (int rc = check_model(m)) return rc;
    const opf::Layout& ly = m->hm.ly;
    int64_t o = 0, l = 0;
    const int64_t P = ly.nrep;
    switch (which) {
    case OPF_VAR_VA: o = ly.x_va; l = ly.N * P; break;
    case OPF_VAR_VM: o = ly.x_vm; l = ly.N * P; break;
    case OPF_VAR_PG: o = ly.x_pg; l = (int64_t)ly.G * ly.npg; break;
    case OPF_VAR_QG: o = ly.x_qg; l = ly.G * P; break;
    case OPF_VAR_P: o = ly.x_p; l = 2LL * ly.L * P; break;
    case OPF_VAR_Q: o = ly.x_q; l = 2LL * ly.L * P; break;
    case OPF_VAR_PS: o = ly.x_ps; l = (int64_t)ly.S * P; break;
    case OPF_VAR_QS: o = ly.x_qs; l = (int64_t)ly.S * P; break;
    case OPF_VAR_QSC: o = ly.x_qsc; l = (int64_t)ly.S * P; break;
    case OPF_VAR_SE: o = ly.x_se; l = (int64_t)ly.S * P; break;
    case OPF_VAR_SC: o = ly.x_sc; l = (int64_t)ly.S * P; break;
    case OPF_VAR_SD: o = ly.x_sd; l = (int64_t)ly.S * P; break;
    case OPF_VAR_U: o = ly.x_u; l = (int64_t)ly.D * P; break;
    default: {
        using namespace opf;
        // OPF_CON_* ids in header order -> constraint blocks
        static const int kBlk[] = {B_REF, B_PFR, B_QFR, B_PTO, B_QTO, B_ANG, B_BALP, B_BALQ, B_THF, B_THT, B_RAMP,
                                   B_ANGL, B_VMAG, B_SOC, B_SLP, B_SLQ, B_STH, B_SCMP, B_DRAMP, B_DINIT};
        if (which >= OPF_CON_REF && which <= OPF_CON_DEV_INIT) {
            const int b = kBlk[which - OPF_CON_REF];
            o = ly.c_blk[b];
            l = ly.c_blk[b + 1] - ly.c_blk[b];
        } else {
            return set_err(OPF_E_ARG, "unknown block id %d", which);
        }
    }
    }
    if (offset) *offset = o;
    if (len) *len = l;
    return OPF_OK;
}

int opf_bounds(opf_model m, double* lvar, double* uvar, double* lcon, double* ucon, double* x0, void* stream) {
    if (int rc = check_model(m)) return rc;
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) return hip_err(dg.err, "hipSetDevice");
    const size_t n = sizeof(double) * m->hm.ly.n, mm = sizeof(double) * m->hm.ly.m();
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::tuple<double*, const double*, size_t> cp[] = {
        {lvar, m->lvar, n}, {uvar, m->uvar, n}, {lcon, m->lcon, mm}, {ucon, m->ucon, mm}, {x0, m->x0, n}};
    for (const auto& c : cp)
        if (std::get<0>(c) && std::get<2>(c)) {
            hipError_t e = hipMemcpyAsync(std::get<0>(c), std::get<1>(c), std::get<2>(c), hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_err(e, "bounds copy");
        }
    return OPF_OK;
}

int opf_obj(opf_model m, const double* x, double* f, void* stream) {
    if (int rc = check_model(m)) return rc;
    if (!x || !f) return set_err(OPF_E_ARG, "x and f must be non-NULL");
    opf::EvalOut o{};
    o.x = x;
    o.f = f;
    return launch_set(m, o, stream);
}

int opf_grad(opf_model m, const double* x, double* g, void* stream) {
    if (int rc = check_model(m)) return rc;
    if (!x || !g) return set_err(OPF_E_ARG, "x and g must be non-NULL");
    opf::EvalOut o{};
    o.x = x;
    o.g = g;
    return launch_set(m, o, stream);
}

int opf_cons(opf_model m, const double* x, double* c, void* stream) {
    if (int rc = check_model(m)) return rc;
    if (!x || !c) return set_err(OPF_E_ARG, "x and c must be non-NULL");
    opf::EvalOut o{};
    o.x = x;
    o.c = c;
    return launch_set(m, o, stream);
}

int opf_jac_structure(opf_model m, int32_t* rows, int32_t* cols, void* stream) {
    if (int rc = check_model(m)) return rc;
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) return hip_err(dg.err, "hipSetDevice");
    const size_t b = sizeof(int32_t) * m->hm.ly.nnzj();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (rows && b) {
        hipError_t e = hipMemcpyAsync(rows, m->jrow, b, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_err(e, "structure copy");
    }
    if (cols && b) {
        hipError_t e = hipMemcpyAsync(cols, m->jcol, b, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_err(e, "structure copy");
    }
    return OPF_OK;
}

int opf_hess_structure(opf_model m, int32_t* rows, int32_t* cols, void* stream) {
    if (int rc = check_model(m)) return rc;
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) return hip_err(dg.err, "hipSetDevice");
    const size_t b = sizeof(int32_t) * m->hm.ly.nnzh;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (rows && b) {
        hipError_t e = hipMemcpyAsync(rows, m->hrow, b, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_err(e, "structure copy");
    }
    if (cols && b) {
        hipError_t e = hipMemcpyAsync(cols, m->hcol, b, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_err(e, "structure copy");
    }
    return OPF_OK;
}

int opf_jac_coord(opf_model m, const double* x, double* vals, void* stream) {
    if (int rc = check_model(m)) return rc;
    if (!x || !vals) return set_err(OPF_E_ARG, "x and vals must be non-NULL");
    opf::EvalOut o{};
    o.x = x;
    o.J = vals;
    return launch_set(m, o, stream);
}

int opf_hess_coord(opf_model m, const double* x, const double* y, double obj_weight, double* vals, void* stream) {
    if (int rc = check_model(m)) return rc;
    if (!x || !y || !vals) return set_err(OPF_E_ARG, "x, y and vals must be non-NULL");
    opf::EvalOut o{};
    o.x = x;
    o.y = y;
    o.sigma = obj_weight;
    o.H = vals;
    return launch_set(m, o, stream);
}

int opf_eval_set(opf_model m, const double* x, const double* y, double obj_weight, double* f, double* g, double* c,
                 double* jvals, double* hvals, void* stream) {
    if (int rc = check_model(m)) return rc;
    if (!x) return set_err(OPF_E_ARG, "x must be non-NULL");
    if (hvals && !y) return set_err(OPF_E_ARG, "y must be non-NULL when hvals is requested");
    opf::EvalOut o{};
    o.x = x;
    o.y = y;
    o.sigma = obj_weight;
    o.f = f;
    o.g = g;
    o.c = c;
    o.J = jvals;
    o.H = hvals;
    return launch_set(m, o, stream);
}

int opf_jtprod(opf_model m, const double* x, const double* v, double* out, void* stream) {
    if (int rc = check_model(m)) return rc;
    if (!x || !v || !out) return set_err(OPF_E_ARG, "x, v and out must be non-NULL");
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) return hip_err(dg.err, "hipSetDevice");
    hipError_t e = opf::launch_jtprod(m->dm, x, v, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_err(e, "jtprod kernel launch");
    return OPF_OK;
}

}  // extern "C"
