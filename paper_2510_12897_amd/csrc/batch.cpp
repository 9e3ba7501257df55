// C-ABI of libopf: batched evaluation of many instances in one persistent
// kernel launch replayed from a HIP graph, with a schedule autotuner.
//
// A schedule is (tile capacity, workgroups per compute unit).  The tile
// capacity fixes which consecutive buses share a workgroup; the workgroup
// count fixes how many persistent workgroups drain the queue.  Neither
// changes any summation order (per-bus sums run over the bus's half-edges in
// their fixed order, the objective over a fixed 256-lane tree), so every
// schedule produces bitwise the same results as the plain per-instance
// launch.
#include <map>
#include <new>
#include <tuple>

#include "internal.h"

using namespace opf_internal;

namespace {

const int32_t kCaps[] = {128, 256, 512, 1024};
const int32_t kWgPerCu[] = {1, 2, 4, 8};

struct Sched {
    int32_t cap = 0;               // effective tile capacity
    opf::BatchInst* inst = nullptr;  // device [n_inst]
    opf::BatchItem* items_eval = nullptr;  // device
    opf::BatchItem* items_jt = nullptr;    // device
    int32_t n_eval = 0, n_jt = 0;
    size_t lds = 0;
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    opf::BatchArgs args{};
};

using GraphKey = std::tuple<int, int32_t, int32_t, const void*, const void*, const void*, const void*, const void*,
                            const void*, const void*, const void*>;

}  // namespace

struct opf_batch_s {
    uint64_t magic = kBatchMagic;
    int device = 0;
    Allocator alloc{};
    int32_t n_inst = 0;
    std::vector<int64_t> xoff, coff, joff, hoff;
    void* arena = nullptr;
    int32_t* counters = nullptr;
    std::vector<Sched> scheds;
    int sched = 0;
    int32_t wg_per_cu = 4;
    int32_t n_cu = 256;
    std::map<GraphKey, GraphEntry> graphs;
};

namespace {

bool valid(const opf_batch_s* b) { return b && b->magic == kBatchMagic; }

void drop_graphs(opf_batch_s* b) {
    for (auto& kv : b->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    b->graphs.clear();
}

// Work items of one schedule: the objective reductions first (long, serial),
// then the bus tiles, branch blocks and generator blocks of every instance.
void make_items(const std::vector<opf::DevModel>& dms, std::vector<opf::BatchItem>& ev,
                std::vector<opf::BatchItem>& jt) {
    ev.clear();
    jt.clear();
    const int32_t n = (int32_t)dms.size();
    for (int32_t j = 0; j < n; j++) ev.push_back({j, opf::T_OBJ, 0, 0});
    for (int32_t j = 0; j < n; j++)
        for (int32_t r = 0; r < dms[j].nrep; r++)
            for (int32_t t = 0; t < dms[j].ntiles; t++) jt.push_back({j, opf::T_BUS, t, r});
    for (int32_t j = 0; j < n; j++) {
        const int32_t nb = (dms[j].L + opf::kBlock - 1) / opf::kBlock;
        for (int32_t r = 0; r < dms[j].nrep; r++)
            for (int32_t t = 0; t < nb; t++) jt.push_back({j, opf::T_BRANCH, t, r});
    }
    for (int32_t j = 0; j < n; j++) {
        const int32_t ng = (std::max(dms[j].G, dms[j].R) + opf::kBlock - 1) / opf::kBlock;
        for (int32_t r = 0; r < dms[j].nrep; r++)
            for (int32_t t = 0; t < ng; t++) jt.push_back({j, opf::T_GEN, t, r});
    }
    ev.insert(ev.end(), jt.begin(), jt.end());
}

int launch(opf_batch_s* b, const opf::BatchArgs& a0, hipStream_t stream) {
    const Sched& s = b->scheds[b->sched];
    opf::BatchArgs a = a0;
    a.inst = s.inst;
    a.counters = b->counters;
    if (a.mode == 0) {
        a.items = s.items_eval;
        a.n_items = s.n_eval;
    } else {
        a.items = s.items_jt;
        a.n_items = s.n_jt;
    }
    if (a.n_items == 0) return OPF_OK;
    const int32_t grid = std::max(1, std::min(a.n_items, b->n_cu * b->wg_per_cu));
    GraphKey key{b->sched, grid, a.mode, a.X, a.Y, a.sigma, a.F, a.G, a.C, a.J, a.H};
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        if (b->graphs.size() >= 512) drop_graphs(b);
        GraphEntry ge;
        ge.args = a;
        hipError_t e = hipGraphCreate(&ge.graph, 0);
        if (e != hipSuccess) return hip_err(e, "hipGraphCreate");
        hipKernelNodeParams p{};
        void* params[] = {&ge.args};
        p.func = opf::batch_kernel_fn();
        p.gridDim = dim3(grid);
        p.blockDim = dim3(opf::kBlock);
        p.sharedMemBytes = (unsigned)s.lds;
        p.kernelParams = params;
        p.extra = nullptr;
        hipGraphNode_t node;
        e = hipGraphAddKernelNode(&node, ge.graph, nullptr, 0, &p);
        if (e == hipSuccess) e = hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (ge.graph) (void)hipGraphDestroy(ge.graph);
            return hip_err(e, "batch graph build");
        }
        it = b->graphs.emplace(key, ge).first;
    }
    hipError_t e = hipGraphLaunch(it->second.exec, stream);
    if (e != hipSuccess) return hip_err(e, "hipGraphLaunch");
    return OPF_OK;
}

}  // namespace

extern "C" {

int opf_batch_create(const opf_model* models, int32_t n_models, const int32_t* inst_model, const double* inst_pd,
                     const double* inst_qd, int32_t n_inst, opf_batch* out) {
    if (!out) return set_err(OPF_E_ARG, "out is NULL");
    *out = nullptr;
    if (!models || n_models < 1 || !inst_model || n_inst < 1)
        return set_err(OPF_E_ARG, "models, inst_model and a positive instance count are required");
    if ((inst_pd == nullptr) != (inst_qd == nullptr))
        return set_err(OPF_E_ARG, "inst_pd and inst_qd must both be given or both be NULL");
    for (int32_t k = 0; k < n_models; k++)
        if (!models[k] || models[k]->magic != kModelMagic)
            return set_err(OPF_E_STATE, "model %d is not a valid handle", k);
    const int dev = models[0]->device;
    for (int32_t k = 1; k < n_models; k++)
        if (models[k]->device != dev) return set_err(OPF_E_ARG, "all models must live on one device");
    for (int32_t j = 0; j < n_inst; j++)
        if (inst_model[j] < 0 || inst_model[j] >= n_models)
            return set_err(OPF_E_ARG, "instance %d names model %d, out of range", j, inst_model[j]);

    opf_batch_s* b = nullptr;
    try {
        b = new opf_batch_s();
        b->device = dev;
        b->alloc = current_allocator();
        b->n_inst = n_inst;
        b->xoff.assign(n_inst + 1, 0);
        b->coff.assign(n_inst + 1, 0);
        b->joff.assign(n_inst + 1, 0);
        b->hoff.assign(n_inst + 1, 0);
        for (int32_t j = 0; j < n_inst; j++) {
            const opf::Layout& ly = models[inst_model[j]]->hm.ly;
            b->xoff[j + 1] = b->xoff[j] + ly.n;
            b->coff[j + 1] = b->coff[j] + ly.m();
            b->joff[j + 1] = b->joff[j] + ly.nnzj();
            b->hoff[j + 1] = b->hoff[j] + ly.nnzh;
        }

        // ---- pack: per-instance loads, per-(model, cap) tiles, then per
        // schedule the instance descriptors and item lists
        Packer pk;
        const size_t o_cnt = pk.reserve(2 * sizeof(int32_t));
        std::vector<size_t> o_pd(n_inst, 0), o_qd(n_inst, 0);
        std::vector<int32_t> stride(n_inst, 0);
        if (inst_pd) {
            int64_t off = 0;
            for (int32_t j = 0; j < n_inst; j++) {
                const opf::HostModel& hm = models[inst_model[j]]->hm;
                const int64_t nl = (int64_t)hm.ly.N * (hm.ly.T > 1 ? hm.ly.T : 1);
                o_pd[j] = pk.add(inst_pd + off, sizeof(double) * nl);
                o_qd[j] = pk.add(inst_qd + off, sizeof(double) * nl);
                stride[j] = hm.ly.T > 1 ? hm.ly.N : 0;
                off += nl;
            }
        }
        std::vector<int32_t> caps;
        for (int32_t c : kCaps) {
            int32_t eff = c;
            for (int32_t k = 0; k < n_models; k++) eff = std::max(eff, models[k]->hm.max_degree);
            if (std::find(caps.begin(), caps.end(), eff) == caps.end()) caps.push_back(eff);
        }
        struct Pending {
            std::vector<size_t> tile_off;  // per model
            std::vector<std::vector<int32_t>> tiles;
            size_t inst_off, ev_off, jt_off;
            int32_t n_ev, n_jt;
            std::vector<opf::DevModel> dms;
            std::vector<opf::BatchItem> ev, jt;
        };
        std::vector<Pending> pend(caps.size());
        for (size_t s = 0; s < caps.size(); s++) {
            Pending& P = pend[s];
            P.tiles.resize(n_models);
            P.tile_off.resize(n_models);
            for (int32_t k = 0; k < n_models; k++) {
                P.tiles[k] = opf::build_tiles(models[k]->hm, caps[s]);
                P.tile_off[k] = pk.add(P.tiles[k]);
            }
            P.dms.resize(n_inst);
            for (int32_t j = 0; j < n_inst; j++) {
                opf::DevModel d = models[inst_model[j]]->dm;
                d.ntiles = (int32_t)P.tiles[inst_model[j]].size() - 1;
                d.tile_cap = caps[s];
                P.dms[j] = d;
            }
            make_items(P.dms, P.ev, P.jt);
            P.n_ev = (int32_t)P.ev.size();
            P.n_jt = (int32_t)P.jt.size();
            P.inst_off = pk.reserve(sizeof(opf::BatchInst) * n_inst);
            P.ev_off = pk.add(P.ev);
            P.jt_off = pk.add(P.jt);
        }

        DeviceGuard dg(dev);
        if (dg.err != hipSuccess) {
            delete b;
            return hip_err(dg.err, "hipSetDevice");
        }
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            b->n_cu = ncu;
        b->arena = dev_alloc(b->alloc, pk.buf.size());
        if (!b->arena) {
            delete b;
            return set_err(OPF_E_NOMEM, "device allocation of %zu bytes failed", pk.buf.size());
        }
        char* base = static_cast<char*>(b->arena);
        // fill the instance descriptors now that device addresses are known
        for (size_t s = 0; s < caps.size(); s++) {
            Pending& P = pend[s];
            opf::BatchInst* hi = reinterpret_cast<opf::BatchInst*>(pk.at(P.inst_off));
            for (int32_t j = 0; j < n_inst; j++) {
                opf::BatchInst bi;
                bi.m = P.dms[j];
                bi.m.tile_bus = reinterpret_cast<const int32_t*>(base + P.tile_off[inst_model[j]]);
                if (inst_pd) {
                    bi.m.pd = reinterpret_cast<const double*>(base + o_pd[j]);
                    bi.m.qd = reinterpret_cast<const double*>(base + o_qd[j]);
                    bi.m.load_stride = stride[j];
                }
                bi.xoff = b->xoff[j];
                bi.coff = b->coff[j];
                bi.joff = b->joff[j];
                bi.hoff = b->hoff[j];
                std::memcpy(&hi[j], &bi, sizeof bi);
            }
            Sched sc;
            sc.cap = caps[s];
            sc.inst = reinterpret_cast<opf::BatchInst*>(base + P.inst_off);
            sc.items_eval = reinterpret_cast<opf::BatchItem*>(base + P.ev_off);
            sc.items_jt = reinterpret_cast<opf::BatchItem*>(base + P.jt_off);
            sc.n_eval = P.n_ev;
            sc.n_jt = P.n_jt;
            opf::DevModel probe = P.dms[0];
            probe.tile_cap = caps[s];
            sc.lds = opf::set_lds_bytes(probe);
            b->scheds.push_back(sc);
        }
        std::memset(pk.at(o_cnt), 0, 2 * sizeof(int32_t));
        hipError_t e = hipMemcpy(b->arena, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dev_free(b->alloc, b->arena);
            delete b;
            return hip_err(e, "batch upload");
        }
        b->counters = reinterpret_cast<int32_t*>(base + o_cnt);
        // default schedule: tile capacity 256 (or the smallest that fits)
        b->sched = 0;
        for (size_t s = 0; s < b->scheds.size(); s++)
            if (b->scheds[s].cap >= 256) {
                b->sched = (int)s;
                break;
            }
    } catch (const std::bad_alloc&) {
        delete b;
        return set_err(OPF_E_NOMEM, "host allocation failed");
    }
    *out = b;
    return OPF_OK;
}

int opf_batch_destroy(opf_batch b) {
    if (!b) return OPF_OK;
    if (!valid(b)) return set_err(OPF_E_STATE, "invalid or destroyed batch handle");
    {
        DeviceGuard dg(b->device);
        (void)hipDeviceSynchronize();
        drop_graphs(b);
        dev_free(b->alloc, b->arena);
    }
    b->magic = 0;
    delete b;
    return OPF_OK;
}

int opf_batch_offsets(opf_batch b, int64_t* xoff, int64_t* coff, int64_t* joff, int64_t* hoff) {
    if (!valid(b)) return set_err(OPF_E_STATE, "invalid or destroyed batch handle");
    const size_t n = sizeof(int64_t) * (b->n_inst + 1);
    if (xoff) std::memcpy(xoff, b->xoff.data(), n);
    if (coff) std::memcpy(coff, b->coff.data(), n);
    if (joff) std::memcpy(joff, b->joff.data(), n);
    if (hoff) std::memcpy(hoff, b->hoff.data(), n);
    return OPF_OK;
}

int opf_batch_schedule(opf_batch b, int32_t* tile_cap, int32_t* wg_per_cu) {
    if (!valid(b)) return set_err(OPF_E_STATE, "invalid or destroyed batch handle");
    if (tile_cap) *tile_cap = b->scheds[b->sched].cap;
    if (wg_per_cu) *wg_per_cu = b->wg_per_cu;
    return OPF_OK;
}

int opf_batch_set_schedule(opf_batch b, int32_t tile_cap, int32_t wg_per_cu) {
    if (!valid(b)) return set_err(OPF_E_STATE, "invalid or destroyed batch handle");
    if (wg_per_cu < 1 || wg_per_cu > 64) return set_err(OPF_E_ARG, "wg_per_cu must be in [1, 64]");
    int found = -1;
    for (size_t s = 0; s < b->scheds.size(); s++)
        if (b->scheds[s].cap >= tile_cap) {
            found = (int)s;
            break;
        }
    if (found < 0) found = (int)b->scheds.size() - 1;
    b->sched = found;
    b->wg_per_cu = wg_per_cu;
    return OPF_OK;
}

int opf_batch_eval(opf_batch b, const double* X, const double* Y, const double* sigma, double* F, double* G,
                   double* C, double* J, double* H, void* stream) {
    if (!valid(b)) return set_err(OPF_E_STATE, "invalid or destroyed batch handle");
    if (!X) return set_err(OPF_E_ARG, "X must be non-NULL");
    if (H && (!Y || !sigma)) return set_err(OPF_E_ARG, "Y and sigma must be non-NULL when H is requested");
    DeviceGuard dg(b->device);
    if (dg.err != hipSuccess) return hip_err(dg.err, "hipSetDevice");
    opf::BatchArgs a{};
    a.X = X; a.Y = Y; a.sigma = sigma; a.F = F; a.G = G; a.C = C; a.J = J; a.H = H;
    a.mode = 0;
    return launch(b, a, static_cast<hipStream_t>(stream));
}

int opf_batch_jtprod(opf_batch b, const double* X, const double* V, double* OUT, void* stream) {
    if (!valid(b)) return set_err(OPF_E_STATE, "invalid or destroyed batch handle");
    if (!X || !V || !OUT) return set_err(OPF_E_ARG, "X, V and OUT must be non-NULL");
    DeviceGuard dg(b->device);
    if (dg.err != hipSuccess) return hip_err(dg.err, "hipSetDevice");
    opf::BatchArgs a{};
    a.X = X; a.Y = V; a.G = OUT;
    a.mode = 1;
    return launch(b, a, static_cast<hipStream_t>(stream));
}

int opf_batch_tune(opf_batch b, void* stream) {
    if (!valid(b)) return set_err(OPF_E_STATE, "invalid or destroyed batch handle");
    DeviceGuard dg(b->device);
    if (dg.err != hipSuccess) return hip_err(dg.err, "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = b->xoff.back(), m = b->coff.back(), nj = b->joff.back(), nh = b->hoff.back();
    const size_t bytes = sizeof(double) * (size_t)(2 * n + 2 * m + nj + nh + 2 * b->n_inst);
    void* buf = dev_alloc(b->alloc, bytes);
    if (!buf) return set_err(OPF_E_NOMEM, "tuning buffers (%zu bytes)", bytes);
    double* p = static_cast<double*>(buf);
    double *X = p, *G = X + n, *Y = G + n, *C = Y + m, *J = C + m, *H = J + nj, *sg = H + nh, *F = sg + b->n_inst;
    int rc = OPF_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int keep_sched = b->sched;
    const int32_t keep_wg = b->wg_per_cu;
    float best = 1e30f;
    int best_s = keep_sched;
    int32_t best_wg = keep_wg;
    do {
        hipError_t e = hipMemsetAsync(buf, 0, bytes, s);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) {
            rc = hip_err(e, "tuning setup");
            break;
        }
        for (size_t sc = 0; sc < b->scheds.size() && rc == OPF_OK; sc++) {
            for (int32_t wg : kWgPerCu) {
                b->sched = (int)sc;
                b->wg_per_cu = wg;
                opf::BatchArgs a{};
                a.X = X; a.Y = Y; a.sigma = sg; a.F = F; a.G = G; a.C = C; a.J = J; a.H = H;
                for (int w = 0; w < 2 && rc == OPF_OK; w++) rc = launch(b, a, s);
                if (rc) break;
                (void)hipEventRecord(e0, s);
                const int reps = 5;
                for (int w = 0; w < reps && rc == OPF_OK; w++) rc = launch(b, a, s);
                if (rc) break;
                (void)hipEventRecord(e1, s);
                e = hipEventSynchronize(e1);
                if (e != hipSuccess) {
                    rc = hip_err(e, "tuning run");
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) {
                    best = ms;
                    best_s = (int)sc;
                    best_wg = wg;
                }
            }
        }
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    drop_graphs(b);  // the tuning buffers are about to be freed
    dev_free(b->alloc, buf);
    if (rc) {
        b->sched = keep_sched;
        b->wg_per_cu = keep_wg;
        return rc;
    }
    b->sched = best_s;
    b->wg_per_cu = best_wg;
    return OPF_OK;
}

}  // extern "C"
