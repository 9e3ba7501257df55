// gfx950 kernels for the polar AC-OPF callbacks (f, grad f, c, J, H) and
// the vector-Jacobian product J^T v.
//
// Every output entry is written exactly once by the work item that owns it,
// with no floating-point atomics; every sum runs in an order fixed by the
// model, so a launch shape gives bitwise the same results however its items
// are scheduled (plain grid, flat or persistent batch grid).
//
// Two-launch shape (large models, batches, J^T v): a callback set runs in
// two phases, each a 64-lane-workgroup launch, and each phase writes only
// outputs laid out in its own order, so every store of a wave lands in a few
// contiguous runs (no scattered partial-line writes, which the per-XCD L2s
// would each write back separately):
//  phase 1, branch items (one lane per branch, branch order, so branch data,
//    multipliers and arc variables are read coalesced; only the four bus
//    voltages are gathered): the four flow rows, the angle row and the two
//    thermal rows (c, J), the arc Hessian diagonals, and one 48-byte record
//    per half-edge (the weighted second derivatives of the branch's flow
//    rows and the arc's p, q), written contiguously in branch order;
//    generator items: the gradient, the pg Hessian diagonal, reference and
//    ramp rows, and one objective partial per (chunk, replica);
//  phase 2, bus items: waves of packed bus segments [head, half-edges,
//    generators] (the host packs them so no segment straddles a wave; an
//    8-byte descriptor per lane, and the head lane's per-bus row offsets,
//    shared with its segment by shuffle, give every output position).  Each
//    half-edge lane reads its record (one aligned 48-byte gather), stages it
//    in LDS, and the
//    head lane reduces its segment in order (a segmented reduction) into the
//    balance rows and the bus's Hessian diagonal, while the first half-edge
//    of each neighbour group writes the group's off-diagonal Hessian
//    entries (parallel branches summed); all of these sit in the bus's own
//    Hessian rows.  Buses wider than a wave are reduced by a whole
//    workgroup; the objective item sums the partials in index order.
// Workgroups are dealt to the 8 XCDs round-robin; both launches remap the
// block index so that each XCD takes a contiguous range of work items, and
// the cache lines that neighbouring items share meet in one L2.
//
// One-launch shape (plain sets of small models, which are latency-bound):
// the same items in one launch, dealt round-robin.  Bus half-edge lanes
// recompute their record from x, y and a slot-ordered copy of the branch
// terms instead of reading it, so results agree with the two-launch shape to
// rounding, not bitwise.  The generator chunk whose arrival completes a
// self-resetting ticket sums the objective partials in index order.
//
// Branch flows follow the pi model of the PowerModels formulation the paper
// uses:  F = alpha u^2 + beta w^2 + u w (a cos(th) + b sin(th)),
// u = vm_f, w = vm_t, th = va_f - va_t, with (alpha, beta, a, b) per flow
//   p_fr: (Gff, 0, Gft, Bft)      q_fr: (-Bff, 0, -Bft, Gft)
//   p_to: (0, Gtt, Gtf, -Btf)     q_to: (0, -Btt, -Btf, -Gtf)
// and the flow row is c = p_arc - F.  Derivatives are written out by hand.
#include <hip/hip_runtime.h>

#include "dev_model.h"
#include "eval_kernels.h"

// No floating-point contraction anywhere in these kernels: every multiply
// and add rounds on its own, so an expression gives bitwise the same value
// in every kernel that inlines it (a one-launch set, whose bus lanes
// recompute the branch terms, equals the two-launch set and the batch bit
// for bit), and each operation rounds as in the oracle.
#pragma clang fp contract(off)

namespace opf {

namespace {

// slot kinds (host_model.h)
constexpr int32_t SK_IDLE = 0, SK_HEAD = 1, SK_EDGE = 2, SK_GEN = 3;

struct Coef {
    double Gff, Bff, Gft, Bft, Gtt, Btt, Gtf, Btf;
};

// Element idx of an array whose base is the same for the whole wave (a
// kernel argument plus uniform offsets).  The byte offset is formed in 32
// bits, so the access compiles to the scalar-base + 32-bit vector-offset
// form and a lane keeps one offset register per index instead of a 64-bit
// address per array.  Every per-instance array is below 4 GiB (checked when
// the model is created).
template <class T>
__device__ __forceinline__ T ld(const T* base, uint32_t idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
}
// Outputs are written once and not read again by the set, so their stores
// are non-temporal (streamed past the caches): they no longer evict the
// model's arrays, which every set re-reads, and leave less dirty data to
// write back when the kernel ends (measured on the 10k-bus set: 9.4 ->
// 8.4 us).  Scratch that a later launch of the same set reads (the
// half-edge records) takes the cached store, st_keep.
template <class T>
__device__ __forceinline__ void st(T* base, uint32_t idx, T v) {
    T* p = reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
    if constexpr (sizeof(T) == 16) {
        typedef double d2v __attribute__((ext_vector_type(2)));
        d2v w;
        __builtin_memcpy(&w, &v, 16);
        __builtin_nontemporal_store(w, reinterpret_cast<d2v*>(p));
    } else {
        __builtin_nontemporal_store(v, p);
    }
}
template <class T>
__device__ __forceinline__ void st_keep(T* base, uint32_t idx, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T))) = v;
}
// Store with the policy chosen at compile time (NT: non-temporal).
template <bool NT, class T>
__device__ __forceinline__ void st_sel(T* base, uint32_t idx, T v) {
    if constexpr (NT)
        st(base, idx, v);
    else
        st_keep(base, idx, v);
}

__device__ __forceinline__ Coef load_coef(const DevModel& m, uint32_t l) {
    const int64_t L = m.L;
    const double* c = m.coef;
    return Coef{ld(c, l),         ld(c + L, l),     ld(c + 2 * L, l), ld(c + 3 * L, l),
                ld(c + 4 * L, l), ld(c + 5 * L, l), ld(c + 6 * L, l), ld(c + 7 * L, l)};
}

// A branch out of service in a contingency copy has zero admittance terms.
__device__ __forceinline__ Coef in_service(const Coef& k, const DevModel& m, int32_t l, int32_t r) {
    return m.outage[r] == l ? Coef{0, 0, 0, 0, 0, 0, 0, 0} : k;
}

// Half-edge records of one side (0: from bus, 1: to bus) and replica r:
// one record per branch (48 bytes, or 16 without the Hessian), branches in
// order; the two sides are separate arrays, so one wave writes each side as
// one contiguous run.
__device__ __forceinline__ double* rec_side(const DevModel& m, int32_t r, int32_t side) {
    return m.rec + ((int64_t)side * m.nrep + r) * m.L * kRecStride;
}
// The J^T v records: two doubles (va term, vm term) per branch and side.
__device__ __forceinline__ double* jt_rec_side(const DevModel& m, int32_t r, int32_t side) {
    return m.rec + ((int64_t)side * m.nrep + r) * m.L * 2;
}

// Store PER values of every lane of a chunk as one contiguous run of
// PER * nvalid doubles starting at dst[first]: staged through LDS, so every
// store instruction of the wave covers consecutive addresses (a lane's own
// values are PER doubles apart, which would touch PER times more cache
// lines per instruction).  KEEP selects the cached store (scratch read by a
// later launch).  Every lane of the workgroup must call it.
template <int PER, bool KEEP = false>
__device__ __forceinline__ void store_run(double* stage, double* dst, uint32_t first, uint32_t nvalid,
                                          const double (&v)[PER]) {
    const uint32_t lane = threadIdx.x;
#pragma unroll
    for (int k = 0; k < PER; k++) stage[PER * lane + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const uint32_t e = k * kBlock + lane;
        if (e < PER * nvalid) {
            if constexpr (KEEP)
                st_keep(dst, first + e, stage[e]);
            else
                st(dst, first + e, stage[e]);
        }
    }
    __syncthreads();
}

// Block index -> work item, so that each XCD (blocks b with b % kXcd equal)
// takes one contiguous range of the nb items.
__device__ __forceinline__ int32_t xcd_item(int32_t b, int32_t nb) {
    const int32_t q = nb / kXcd, rem = nb % kXcd;
    const int32_t x = b % kXcd, j = b / kXcd;
    return x * q + min(x, rem) + j;
}

// Sum over the wave in a fixed tree order; lane 0 holds the total.
__device__ __forceinline__ double wave_sum(double v) {
    for (int s = kBlock / 2; s > 0; s >>= 1) v += __shfl_down(v, s, kBlock);
    return v;
}

// First-order terms of one flow F = al u^2 + be w^2 + u w (a C + b S).
struct Flow1 {
    double F, Fu, Fw, Ft;
};
__device__ __forceinline__ Flow1 flow1(double al, double be, double a, double b, double u, double w, double C,
                                       double S) {
    const double k1 = a * C + b * S;
    const double k2 = b * C - a * S;
    const double uw = u * w;
    Flow1 r;
    r.F = al * u * u + be * w * w + uw * k1;
    r.Fu = 2.0 * al * u + w * k1;
    r.Fw = 2.0 * be * w + u * k1;
    r.Ft = uw * k2;
    return r;
}

// Second-order terms of sum_r (-y_r) F_r over the four flow rows of a branch
// (each row is p_arc - F_r).  hess F is linear in (alpha, beta, a, b), so the
// weighted sum needs one trig evaluation.  The branch items (records) and
// the one-launch bus lanes (recompute) both call it.
struct Hterms {
    double Suu, Sww, Suw, Stt, Sut, Swt;  // d2/du2, dw2, du dw, dth2, du dth, dw dth
};
__device__ __forceinline__ Hterms hess_terms(const Coef& k, double y1, double y2, double y3, double y4, double u,
                                             double w, double C, double S) {
    const double Wal = -(y1 * k.Gff - y2 * k.Bff);
    const double Wbe = -(y3 * k.Gtt - y4 * k.Btt);
    const double A = -(y1 * k.Gft - y2 * k.Bft + y3 * k.Gtf - y4 * k.Btf);
    const double B = -(y1 * k.Bft + y2 * k.Gft - y3 * k.Btf - y4 * k.Gtf);
    const double K1 = A * C + B * S, K2 = B * C - A * S;
    Hterms h;
    h.Suu = 2.0 * Wal;
    h.Sww = 2.0 * Wbe;
    h.Suw = K1;
    h.Stt = -u * w * K1;
    h.Sut = w * K2;
    h.Swt = u * K2;
    return h;
}

// sum_r v_r dc_r/d(th, u, w) over the four flow rows (c = p_arc - F).
struct Jterms {
    double Dt, Du, Dw;
};
__device__ __forceinline__ Jterms jt_terms(const Coef& k, double v1, double v2, double v3, double v4, double u,
                                           double w, double C, double S) {
    const double Wal = v1 * k.Gff - v2 * k.Bff;
    const double Wbe = v3 * k.Gtt - v4 * k.Btt;
    const double A = v1 * k.Gft - v2 * k.Bft + v3 * k.Gtf - v4 * k.Btf;
    const double B = v1 * k.Bft + v2 * k.Gft - v3 * k.Btf - v4 * k.Gtf;
    const double K1 = A * C + B * S, K2 = B * C - A * S;
    Jterms j;
    j.Dt = -u * w * K2;
    j.Du = -(2.0 * Wal * u + w * K1);
    j.Dw = -(2.0 * Wbe * w + u * K1);
    return j;
}

// The five Jacobian entries of one flow row, columns in ascending order:
// the lower bus's va, the higher bus's va, then the vm pair, then the arc
// variable.
__device__ __forceinline__ void flow_jrow(const Flow1& fl, bool f_lo, double (&v)[5]) {
    v[0] = f_lo ? -fl.Ft : fl.Ft;
    v[1] = f_lo ? fl.Ft : -fl.Ft;
    v[2] = f_lo ? -fl.Fu : -fl.Fw;
    v[3] = f_lo ? -fl.Fw : -fl.Fu;
    v[4] = 1.0;
}

// The half-edge record [TT, MA, MM, UW, P, Q] of branch l at one side (0:
// from, 1: to), recomputed from x and y with the branch task's arithmetic:
// a single launch reads nothing the branch items write.  Split into its
// loads and its arithmetic so that a wave can issue the loads of all its
// lane types before it waits for any.
struct HeIn {
    double p, q, y1, y2, y3, y4, u, w, vaf, vat;
};
__device__ __forceinline__ void half_edge_load(const DevModel& m, const EvalOut& o, uint32_t l, uint32_t side,
                                               uint32_t fb, uint32_t tb, int32_t r, HeIn& e) {
    const int64_t L = m.L, N = m.N, ob = L * r, oa = 2 * L * r + (side ? L : 0), on = N * r;
    if (o.c) {
        e.p = ld(o.x + m.x_p + oa, l);
        e.q = ld(o.x + m.x_q + oa, l);
    }
    if (o.H) {
        e.y1 = ld(o.y + m.c_pfr + ob, l);
        e.y2 = ld(o.y + m.c_qfr + ob, l);
        e.y3 = ld(o.y + m.c_pto + ob, l);
        e.y4 = ld(o.y + m.c_qto + ob, l);
        e.u = ld(o.x + m.x_vm + on, fb);
        e.w = ld(o.x + m.x_vm + on, tb);
        e.vaf = ld(o.x + m.x_va + on, fb);
        e.vat = ld(o.x + m.x_va + on, tb);
    }
}
__device__ __forceinline__ void half_edge_record(const DevModel& m, const EvalOut& o, const HeIn& e, uint32_t l,
                                                 uint32_t side, const Coef& k0, int32_t r, double (&v)[kRec]) {
    if (o.c) {
        v[R_P] = e.p;
        v[R_Q] = e.q;
    }
    if (o.H) {
        const Coef k = in_service(k0, m, (int32_t)l, r);
        double S, C;
        sincos(e.vaf - e.vat, &S, &C);
        const Hterms h = hess_terms(k, e.y1, e.y2, e.y3, e.y4, e.u, e.w, C, S);
        v[R_TT] = h.Stt;
        v[R_MA] = side ? -h.Swt : h.Sut;
        v[R_MM] = side ? h.Sww : h.Suu;
        v[R_UW] = h.Suw;
    }
}

// ------------------------------------------------------- rectangular form
// With V = vr + j vi (Sec. III-C1, form = :rect) the branch rows are
// polynomials: CR = vr_f vr_t + vi_f vi_t and SI = vi_f vr_t - vr_f vi_t
// stand for vm_f vm_t cos(th) and vm_f vm_t sin(th), Uf = |V_f|^2 and
// Ut = |V_t|^2 for vm_f^2 and vm_t^2, so every flow is
//   F = al Uf + be Ut + a CR + b SI
// with the polar (al, be, a, b), and the two angle rows are SI - tan(lim) CR
// (al = be = 0, a = -tan(lim), b = 1).  No trigonometry.
struct RVolt {
    double rf, rt, jf, jt;  // vr_f, vr_t, vi_f, vi_t
};
struct RTerm {
    double F, Drf, Drt, Djf, Djt;  // value and d/d(vr_f, vr_t, vi_f, vi_t)
};
__device__ __forceinline__ RTerm rterm(double al, double be, double a, double b, const RVolt& v, double CR,
                                       double SI, double Uf, double Ut) {
    RTerm r;
    r.F = al * Uf + be * Ut + a * CR + b * SI;
    r.Drf = 2.0 * al * v.rf + a * v.rt - b * v.jt;
    r.Drt = 2.0 * be * v.rt + a * v.rf + b * v.jf;
    r.Djf = 2.0 * al * v.jf + a * v.jt + b * v.rt;
    r.Djt = 2.0 * be * v.jt + a * v.jf - b * v.rf;
    return r;
}
// Jacobian entries of a row with partials t, columns ascending (vr_lo,
// vr_hi, vi_lo, vi_hi, then the arc variable's 1 when NV = 5), scaled by sg
// (-1 for a flow row p - F).
template <int NV>
__device__ __forceinline__ void rect_jrow(const RTerm& t, bool f_lo, double sg, double (&v)[NV]) {
    v[0] = sg * (f_lo ? t.Drf : t.Drt);
    v[1] = sg * (f_lo ? t.Drt : t.Drf);
    v[2] = sg * (f_lo ? t.Djf : t.Djt);
    v[3] = sg * (f_lo ? t.Djt : t.Djf);
    if constexpr (NV == 5) v[4] = 1.0;
}
// The multiplier-weighted sum W = sum_r y_r c_r over a branch's six voltage
// rows (four flows p - F, two angle rows) as W = al Uf + be Ut + A CR + B SI
// (+ the linear arc terms): its second derivatives are d2W/dvr_f2 =
// d2W/dvi_f2 = 2 al, d2W/dvr_t2 = d2W/dvi_t2 = 2 be, d2W/(dvr_f dvr_t) =
// d2W/(dvi_f dvi_t) = A, d2W/(dvi_f dvr_t) = B, d2W/(dvr_f dvi_t) = -B.
struct RW {
    double al, be, A, B;
};
__device__ __forceinline__ RW rect_w(const Coef& k, double t5, double t6, double y1, double y2, double y3, double y4,
                                     double y5, double y6) {
    RW w;
    w.al = -(y1 * k.Gff - y2 * k.Bff);
    w.be = -(y3 * k.Gtt - y4 * k.Btt);
    w.A = -(y1 * k.Gft - y2 * k.Bft + y3 * k.Gtf - y4 * k.Btf) - y5 * t5 - y6 * t6;
    w.B = -(y1 * k.Bft + y2 * k.Gft - y3 * k.Btf - y4 * k.Gtf) + y5 + y6;
    return w;
}
// The rectangular half-edge record [D, Bs, D, A, P, Q] of one side (own
// bus i, other bus k): D = the (vr_i, vr_i) and (vi_i, vi_i) term, Bs = the
// (vi_i, vr_k) term, A = the (vr_i, vr_k) and (vi_i, vi_k) term; the fields
// sit where the bus phase sums the polar record's (TT, MA, MM, UW).
__device__ __forceinline__ void rect_record(const RW& w, uint32_t side, double p, double q, double (&v)[kRec]) {
    v[R_TT] = side ? 2.0 * w.be : 2.0 * w.al;
    v[R_MA] = side ? -w.B : w.B;
    v[R_MM] = v[R_TT];
    v[R_UW] = w.A;
    v[R_P] = p;
    v[R_Q] = q;
}

// The rectangular record of branch l at one side, recomputed from x and y
// (one launch).  Loads first, arithmetic second (as half_edge_load / _record).
struct RHeIn {
    double p, q, y1, y2, y3, y4, y5, y6, t5, t6;
    RVolt v;
};
__device__ __forceinline__ void rect_edge_load(const DevModel& m, const EvalOut& o, uint32_t l, uint32_t side,
                                               uint32_t fb, uint32_t tb, int32_t r, RHeIn& e) {
    const int64_t L = m.L, N = m.N, ob = L * r, oa = 2 * L * r + (side ? L : 0), on = N * r;
    if (o.c) {
        e.p = ld(o.x + m.x_p + oa, l);
        e.q = ld(o.x + m.x_q + oa, l);
    }
    if (o.H) {
        e.y1 = ld(o.y + m.c_pfr + ob, l);
        e.y2 = ld(o.y + m.c_qfr + ob, l);
        e.y3 = ld(o.y + m.c_pto + ob, l);
        e.y4 = ld(o.y + m.c_qto + ob, l);
        e.y5 = ld(o.y + m.c_ang + ob, l);
        e.y6 = ld(o.y + m.c_angl + ob, l);
        e.t5 = ld(m.tan_lim, l);
        e.t6 = ld(m.tan_lim + L, l);
        e.v.rf = ld(o.x + m.x_va + on, fb);
        e.v.rt = ld(o.x + m.x_va + on, tb);
        e.v.jf = ld(o.x + m.x_vm + on, fb);
        e.v.jt = ld(o.x + m.x_vm + on, tb);
    }
}
__device__ __forceinline__ void rect_edge_record(const DevModel& m, const EvalOut& o, const RHeIn& e, uint32_t l,
                                                 uint32_t side, const Coef& k0, int32_t r, double (&v)[kRec]) {
    if (o.H) {
        const Coef k = in_service(k0, m, (int32_t)l, r);
        rect_record(rect_w(k, e.t5, e.t6, e.y1, e.y2, e.y3, e.y4, e.y5, e.y6), side, 0.0, 0.0, v);
    }
    if (o.c) {
        v[R_P] = e.p;
        v[R_Q] = e.q;
    }
}

// The (vm, vm) Hessian term of a storage unit's loss rows at its bus:
// -(y_lp r + y_lq x) d2 i2 / dvm2 with d2 i2 / dvm2 = 6 S2 / vm^4.
__device__ __forceinline__ double stor_vmvm(double ps, double qs, double vm, double ylp, double ylq, double rr,
                                            double xx) {
    const double iv2 = 1.0 / (vm * vm);
    return -(ylp * rr + ylq * xx) * 6.0 * (ps * ps + qs * qs) * iv2 * iv2;
}

// The vm entry of J^T v from a storage unit's loss rows:
// (v_lp r + v_lq x) 2 S2 / vm^3.
__device__ __forceinline__ double jt_stor_vm(double ps, double qs, double vm, double vlp, double vlq, double rr,
                                             double xx) {
    return (vlp * rr + vlq * xx) * 2.0 * (ps * ps + qs * qs) / (vm * vm * vm);
}

// ================================================================== phase 1
template <bool SINGLE>
__device__ void branch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r, double* stage) {
    const uint32_t l0 = (uint32_t)(chunk * kBlock), l = l0 + threadIdx.x;
    const uint32_t nvalid = min((uint32_t)kBlock, (uint32_t)m.L - l0);
    const bool act = l < (uint32_t)m.L;  // inactive lanes still join the LDS staging
    const int64_t L = m.L, N = m.N;
    const bool wantC = o.c != nullptr, wantJ = o.J != nullptr, wantH = o.H != nullptr;
    const int64_t ob = L * r;       // branch blocks of replica r
    const int64_t oa = 2 * L * r;   // arc blocks of replica r (from arcs, then to arcs)
    const int64_t on = N * r;       // bus blocks of replica r
    if (wantC || wantJ || wantH) {
        // every load before the first store: loads and stores share one
        // in-order completion counter, so a load issued after stores would
        // also wait for all of them to complete
        uint32_t fb = 0, tb = 0;
        double rate2 = 0.0, pf = 0.0, pt = 0.0, qf = 0.0, qt = 0.0;
        double yf = 0.0, yt = 0.0, y1 = 0.0, y2 = 0.0, y3 = 0.0, y4 = 0.0;
        double u = 1.0, w = 1.0, vaf = 0.0, vat = 0.0;
        Coef k{};
        if (act) {
            fb = (uint32_t)ld(m.f_bus, l);
            tb = (uint32_t)ld(m.t_bus, l);
            k = in_service(load_coef(m, l), m, (int32_t)l, r);
            if (wantC) rate2 = ld(m.rate2, l);
            const double* xp = o.x + m.x_p + oa;
            const double* xq = o.x + m.x_q + oa;
            pf = ld(xp, l);
            pt = ld(xp + L, l);
            qf = ld(xq, l);
            qt = ld(xq + L, l);
            if (wantH) {
                yf = ld(o.y + m.c_thf + ob, l);
                yt = ld(o.y + m.c_tht + ob, l);
                y1 = ld(o.y + m.c_pfr + ob, l);
                y2 = ld(o.y + m.c_qfr + ob, l);
                y3 = ld(o.y + m.c_pto + ob, l);
                y4 = ld(o.y + m.c_qto + ob, l);
            }
            u = ld(o.x + m.x_vm + on, fb);
            w = ld(o.x + m.x_vm + on, tb);
            vaf = ld(o.x + m.x_va + on, fb);
            vat = ld(o.x + m.x_va + on, tb);
        }
        const bool f_lo = fb < tb;
        double S, C;
        sincos(vaf - vat, &S, &C);
        const Flow1 f1 = flow1(k.Gff, 0.0, k.Gft, k.Bft, u, w, C, S);
        const Flow1 f2 = flow1(-k.Bff, 0.0, -k.Bft, k.Gft, u, w, C, S);
        const Flow1 f3 = flow1(0.0, k.Gtt, k.Gtf, -k.Btf, u, w, C, S);
        const Flow1 f4 = flow1(0.0, -k.Btt, -k.Btf, -k.Gtf, u, w, C, S);
        if (wantC && act) {
            st(o.c + m.c_pfr + ob, l, pf - f1.F);
            st(o.c + m.c_qfr + ob, l, qf - f2.F);
            st(o.c + m.c_pto + ob, l, pt - f3.F);
            st(o.c + m.c_qto + ob, l, qt - f4.F);
            st(o.c + m.c_ang + ob, l, vaf - vat);
            st(o.c + m.c_thf + ob, l, pf * pf + qf * qf - rate2);
            st(o.c + m.c_tht + ob, l, pt * pt + qt * qt - rate2);
        }
        if (wantJ) {
            // the flow-row blocks (5 values per lane) go through LDS so that
            // each store instruction of the wave covers consecutive addresses
            // (in the one-launch shape too: 9.75 -> 9.41 us on the 10k-bus
            // set); the 2-value pairs are stored directly, since staging them
            // as well cost more in barriers than it saved (10.4 us)
            double v[5];
            flow_jrow(f1, f_lo, v);
            store_run<5>(stage, o.J + m.j_pfr + 5 * ob, 5 * l0, nvalid, v);
            flow_jrow(f2, f_lo, v);
            store_run<5>(stage, o.J + m.j_qfr + 5 * ob, 5 * l0, nvalid, v);
            flow_jrow(f3, f_lo, v);
            store_run<5>(stage, o.J + m.j_pto + 5 * ob, 5 * l0, nvalid, v);
            flow_jrow(f4, f_lo, v);
            store_run<5>(stage, o.J + m.j_qto + 5 * ob, 5 * l0, nvalid, v);
            if (act) {
                // block offsets need not be even, so these pairs are stored
                // as two 8-byte values
                st(o.J + m.j_ang + 2 * ob, 2 * l, f_lo ? 1.0 : -1.0);
                st(o.J + m.j_ang + 2 * ob, 2 * l + 1, f_lo ? -1.0 : 1.0);
                st(o.J + m.j_thf + 2 * ob, 2 * l, 2.0 * pf);
                st(o.J + m.j_thf + 2 * ob, 2 * l + 1, 2.0 * qf);
                st(o.J + m.j_tht + 2 * ob, 2 * l, 2.0 * pt);
                st(o.J + m.j_tht + 2 * ob, 2 * l + 1, 2.0 * qt);
            }
        }
        if (wantH && act) {
            st(o.H + m.h_p + oa, l, 2.0 * yf);
            st(o.H + m.h_p + oa + L, l, 2.0 * yt);
            st(o.H + m.h_q + oa, l, 2.0 * yf);
            st(o.H + m.h_q + oa + L, l, 2.0 * yt);
        }
        if (wantH && !SINGLE) {
            // the half-edge records [TT, MA, MM, UW, P, Q] of each side
            const Hterms h = hess_terms(k, y1, y2, y3, y4, u, w, C, S);
            // d/dva_f = d/dth, d/dva_t = -d/dth
            const double rf[kRecStride] = {h.Stt, h.Sut, h.Suu, h.Suw, pf, qf};
            store_run<kRecStride, true>(stage, rec_side(m, r, 0), kRecStride * l0, nvalid, rf);
            const double rt[kRecStride] = {h.Stt, -h.Swt, h.Sww, h.Suw, pt, qt};
            store_run<kRecStride, true>(stage, rec_side(m, r, 1), kRecStride * l0, nvalid, rt);
        } else if (wantC && !SINGLE) {
            // no Hessian: compact records [P, Q] (the balance rows need nothing else)
            const double rf[kRecPQ] = {pf, qf};
            store_run<kRecPQ, true>(stage, rec_side(m, r, 0), kRecPQ * l0, nvalid, rf);
            const double rt[kRecPQ] = {pt, qt};
            store_run<kRecPQ, true>(stage, rec_side(m, r, 1), kRecPQ * l0, nvalid, rt);
        }
    }
    if (o.g && act) {
        st(o.g + m.x_p + oa, l, 0.0);
        st(o.g + m.x_p + oa + L, l, 0.0);
        st(o.g + m.x_q + oa, l, 0.0);
        st(o.g + m.x_q + oa + L, l, 0.0);
    }
}

// Phase 1 of the rectangular form: one lane per branch, as branch_task;
// writes the four flow rows, the two angle rows, the two thermal rows, the
// arc Hessian diagonals and the half-edge records [D, Bs, D, A, P, Q].
template <bool SINGLE>
__device__ void rbranch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r, double* stage) {
    const uint32_t l0 = (uint32_t)(chunk * kBlock), l = l0 + threadIdx.x;
    const uint32_t nvalid = min((uint32_t)kBlock, (uint32_t)m.L - l0);
    const bool act = l < (uint32_t)m.L;  // inactive lanes still join the LDS staging
    const int64_t L = m.L, N = m.N;
    const bool wantC = o.c != nullptr, wantJ = o.J != nullptr, wantH = o.H != nullptr;
    const int64_t ob = L * r, oa = 2 * L * r, on = N * r;
    if (wantC || wantJ || wantH) {
        uint32_t fb = 0, tb = 0;
        double rate2 = 0.0, pf = 0.0, pt = 0.0, qf = 0.0, qt = 0.0, t5 = 0.0, t6 = 0.0;
        double yf = 0.0, yt = 0.0, y1 = 0.0, y2 = 0.0, y3 = 0.0, y4 = 0.0, y5 = 0.0, y6 = 0.0;
        RVolt v{1.0, 1.0, 0.0, 0.0};
        Coef k{};
        if (act) {
            fb = (uint32_t)ld(m.f_bus, l);
            tb = (uint32_t)ld(m.t_bus, l);
            k = in_service(load_coef(m, l), m, (int32_t)l, r);
            if (wantC) rate2 = ld(m.rate2, l);
            t5 = ld(m.tan_lim, l);
            t6 = ld(m.tan_lim + L, l);
            const double* xp = o.x + m.x_p + oa;
            const double* xq = o.x + m.x_q + oa;
            pf = ld(xp, l);
            pt = ld(xp + L, l);
            qf = ld(xq, l);
            qt = ld(xq + L, l);
            if (wantH) {
                yf = ld(o.y + m.c_thf + ob, l);
                yt = ld(o.y + m.c_tht + ob, l);
                y1 = ld(o.y + m.c_pfr + ob, l);
                y2 = ld(o.y + m.c_qfr + ob, l);
                y3 = ld(o.y + m.c_pto + ob, l);
                y4 = ld(o.y + m.c_qto + ob, l);
                y5 = ld(o.y + m.c_ang + ob, l);
                y6 = ld(o.y + m.c_angl + ob, l);
            }
            v.rf = ld(o.x + m.x_va + on, fb);
            v.rt = ld(o.x + m.x_va + on, tb);
            v.jf = ld(o.x + m.x_vm + on, fb);
            v.jt = ld(o.x + m.x_vm + on, tb);
        }
        const bool f_lo = fb < tb;
        const double CR = v.rf * v.rt + v.jf * v.jt, SI = v.jf * v.rt - v.rf * v.jt;
        const double Uf = v.rf * v.rf + v.jf * v.jf, Ut = v.rt * v.rt + v.jt * v.jt;
        const RTerm f1 = rterm(k.Gff, 0.0, k.Gft, k.Bft, v, CR, SI, Uf, Ut);
        const RTerm f2 = rterm(-k.Bff, 0.0, -k.Bft, k.Gft, v, CR, SI, Uf, Ut);
        const RTerm f3 = rterm(0.0, k.Gtt, k.Gtf, -k.Btf, v, CR, SI, Uf, Ut);
        const RTerm f4 = rterm(0.0, -k.Btt, -k.Btf, -k.Gtf, v, CR, SI, Uf, Ut);
        const RTerm a5 = rterm(0.0, 0.0, -t5, 1.0, v, CR, SI, Uf, Ut);
        const RTerm a6 = rterm(0.0, 0.0, -t6, 1.0, v, CR, SI, Uf, Ut);
        if (wantC && act) {
            st(o.c + m.c_pfr + ob, l, pf - f1.F);
            st(o.c + m.c_qfr + ob, l, qf - f2.F);
            st(o.c + m.c_pto + ob, l, pt - f3.F);
            st(o.c + m.c_qto + ob, l, qt - f4.F);
            st(o.c + m.c_ang + ob, l, a5.F);
            st(o.c + m.c_angl + ob, l, a6.F);
            st(o.c + m.c_thf + ob, l, pf * pf + qf * qf - rate2);
            st(o.c + m.c_tht + ob, l, pt * pt + qt * qt - rate2);
        }
        if (wantJ) {
            // flow rows (vr_lo, vr_hi, vi_lo, vi_hi, arc) and angle rows
            // (vr_lo, vr_hi, vi_lo, vi_hi), staged through LDS
            double v5[5], v4[4];
            rect_jrow(f1, f_lo, -1.0, v5);
            store_run<5>(stage, o.J + m.j_pfr + 5 * ob, 5 * l0, nvalid, v5);
            rect_jrow(f2, f_lo, -1.0, v5);
            store_run<5>(stage, o.J + m.j_qfr + 5 * ob, 5 * l0, nvalid, v5);
            rect_jrow(f3, f_lo, -1.0, v5);
            store_run<5>(stage, o.J + m.j_pto + 5 * ob, 5 * l0, nvalid, v5);
            rect_jrow(f4, f_lo, -1.0, v5);
            store_run<5>(stage, o.J + m.j_qto + 5 * ob, 5 * l0, nvalid, v5);
            rect_jrow(a5, f_lo, 1.0, v4);
            store_run<4>(stage, o.J + m.j_ang + 4 * ob, 4 * l0, nvalid, v4);
            rect_jrow(a6, f_lo, 1.0, v4);
            store_run<4>(stage, o.J + m.j_angl + 4 * ob, 4 * l0, nvalid, v4);
            if (act) {
                st(o.J + m.j_thf + 2 * ob, 2 * l, 2.0 * pf);
                st(o.J + m.j_thf + 2 * ob, 2 * l + 1, 2.0 * qf);
                st(o.J + m.j_tht + 2 * ob, 2 * l, 2.0 * pt);
                st(o.J + m.j_tht + 2 * ob, 2 * l + 1, 2.0 * qt);
            }
        }
        if (wantH && act) {
            st(o.H + m.h_p + oa, l, 2.0 * yf);
            st(o.H + m.h_p + oa + L, l, 2.0 * yt);
            st(o.H + m.h_q + oa, l, 2.0 * yf);
            st(o.H + m.h_q + oa + L, l, 2.0 * yt);
        }
        if (wantH && !SINGLE) {
            const RW w = rect_w(k, t5, t6, y1, y2, y3, y4, y5, y6);
            double rf[kRec], rt[kRec];
            rect_record(w, 0, pf, qf, rf);
            rect_record(w, 1, pt, qt, rt);
            store_run<kRecStride, true>(stage, rec_side(m, r, 0), kRecStride * l0, nvalid, rf);
            store_run<kRecStride, true>(stage, rec_side(m, r, 1), kRecStride * l0, nvalid, rt);
        } else if (wantC && !SINGLE) {
            const double rf[kRecPQ] = {pf, qf};
            store_run<kRecPQ, true>(stage, rec_side(m, r, 0), kRecPQ * l0, nvalid, rf);
            const double rt[kRecPQ] = {pt, qt};
            store_run<kRecPQ, true>(stage, rec_side(m, r, 1), kRecPQ * l0, nvalid, rt);
        }
    }
    if (o.g && act) {
        st(o.g + m.x_p + oa, l, 0.0);
        st(o.g + m.x_p + oa + L, l, 0.0);
        st(o.g + m.x_q + oa, l, 0.0);
        st(o.g + m.x_q + oa + L, l, 0.0);
    }
}

// J^T v of the rectangular form, phase 1: the arc entries (as polar) and
// each half-edge's (vr, vi) terms: the gradient of W = sum_r v_r c_r over
// the branch's six voltage rows at the side's own bus.
__device__ void rjt_branch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const uint32_t l = (uint32_t)(chunk * kBlock) + threadIdx.x;
    if (l >= (uint32_t)m.L) return;
    const int64_t L = m.L, N = m.N;
    const uint32_t fb = (uint32_t)ld(m.f_bus, l), tb = (uint32_t)ld(m.t_bus, l);
    const Coef k0 = load_coef(m, l);
    const double t5 = ld(m.tan_lim, l), t6 = ld(m.tan_lim + L, l);
    const double* x = o.x;
    const double* v = o.y;
    const int64_t ob = L * r, oa = 2 * L * r, on = N * r;
    const double vtf = ld(v + m.c_thf + ob, l), vtt = ld(v + m.c_tht + ob, l);
    const double v1 = ld(v + m.c_pfr + ob, l), v2 = ld(v + m.c_qfr + ob, l);
    const double v3 = ld(v + m.c_pto + ob, l), v4 = ld(v + m.c_qto + ob, l);
    const double v5 = ld(v + m.c_ang + ob, l), v6 = ld(v + m.c_angl + ob, l);
    const double pf = ld(x + m.x_p + oa, l), pt = ld(x + m.x_p + oa + L, l);
    const double qf = ld(x + m.x_q + oa, l), qt = ld(x + m.x_q + oa + L, l);
    const double bpf = ld(v + m.c_balp + on, fb), bpt = ld(v + m.c_balp + on, tb);
    const double bqf = ld(v + m.c_balq + on, fb), bqt = ld(v + m.c_balq + on, tb);
    RVolt e;
    e.rf = ld(x + m.x_va + on, fb);
    e.rt = ld(x + m.x_va + on, tb);
    e.jf = ld(x + m.x_vm + on, fb);
    e.jt = ld(x + m.x_vm + on, tb);
    const Coef k = in_service(k0, m, (int32_t)l, r);
    st(o.g + m.x_p + oa, l, v1 + bpf + 2.0 * pf * vtf);
    st(o.g + m.x_p + oa + L, l, v3 + bpt + 2.0 * pt * vtt);
    st(o.g + m.x_q + oa, l, v2 + bqf + 2.0 * qf * vtf);
    st(o.g + m.x_q + oa + L, l, v4 + bqt + 2.0 * qt * vtt);
    const RW w = rect_w(k, t5, t6, v1, v2, v3, v4, v5, v6);
    const double CR = 0.0, SI = 0.0;
    const RTerm d = rterm(w.al, w.be, w.A, w.B, e, CR, SI, 0.0, 0.0);
    st_keep(reinterpret_cast<double2*>(jt_rec_side(m, r, 0)), l, make_double2(d.Drf, d.Djf));
    st_keep(reinterpret_cast<double2*>(jt_rec_side(m, r, 1)), l, make_double2(d.Drt, d.Djt));
}

// J^T v, phase 1: the arc entries p / q (owned here) and each half-edge's
// va / vm terms for the bus side.
__device__ void jt_branch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const uint32_t l = (uint32_t)(chunk * kBlock) + threadIdx.x;
    if (l >= (uint32_t)m.L) return;
    const int64_t L = m.L, N = m.N;
    const uint32_t fb = (uint32_t)ld(m.f_bus, l), tb = (uint32_t)ld(m.t_bus, l);
    const Coef k0 = load_coef(m, l);
    const double* x = o.x;
    const double* v = o.y;
    {  // replica r
        const int64_t ob = L * r, oa = 2 * L * r, on = N * r;
        // every load before the first store (one in-order completion counter)
        const double vtf = ld(v + m.c_thf + ob, l), vtt = ld(v + m.c_tht + ob, l);
        const double v1 = ld(v + m.c_pfr + ob, l), v2 = ld(v + m.c_qfr + ob, l);
        const double v3 = ld(v + m.c_pto + ob, l), v4 = ld(v + m.c_qto + ob, l);
        const double va = ld(v + m.c_ang + ob, l);
        const double pf = ld(x + m.x_p + oa, l), pt = ld(x + m.x_p + oa + L, l);
        const double qf = ld(x + m.x_q + oa, l), qt = ld(x + m.x_q + oa + L, l);
        const double bpf = ld(v + m.c_balp + on, fb), bpt = ld(v + m.c_balp + on, tb);
        const double bqf = ld(v + m.c_balq + on, fb), bqt = ld(v + m.c_balq + on, tb);
        const double u = ld(x + m.x_vm + on, fb), w = ld(x + m.x_vm + on, tb);
        const double th = ld(x + m.x_va + on, fb) - ld(x + m.x_va + on, tb);
        const Coef k = in_service(k0, m, (int32_t)l, r);
        // p_a sits in its flow row (+1), its bus's balance row (+1) and its
        // thermal row (2 p_a); q_a likewise
        st(o.g + m.x_p + oa, l, v1 + bpf + 2.0 * pf * vtf);
        st(o.g + m.x_p + oa + L, l, v3 + bpt + 2.0 * pt * vtt);
        st(o.g + m.x_q + oa, l, v2 + bqf + 2.0 * qf * vtf);
        st(o.g + m.x_q + oa + L, l, v4 + bqt + 2.0 * qt * vtt);
        double S, C;
        sincos(th, &S, &C);
        const Jterms j = jt_terms(k, v1, v2, v3, v4, u, w, C, S);
        // d th / d va_f = 1, d th / d va_t = -1; the angle row is va_f - va_t
        st_keep(reinterpret_cast<double2*>(jt_rec_side(m, r, 0)), l, make_double2(j.Dt + va, j.Du));
        st_keep(reinterpret_cast<double2*>(jt_rec_side(m, r, 1)), l, make_double2(-j.Dt - va, j.Dw));
    }
}

// Arc variables := branch flows F(vm, va) (the x rows are read from o.x,
// the p / q entries written through o.g, which may alias it).
__device__ void flows_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const uint32_t l = (uint32_t)(chunk * kBlock) + threadIdx.x;
    if (l >= (uint32_t)m.L) return;
    const int64_t L = m.L, N = m.N;
    const uint32_t fb = (uint32_t)ld(m.f_bus, l), tb = (uint32_t)ld(m.t_bus, l);
    const Coef k0 = load_coef(m, l);
    {  // replica r
        const int64_t oa = 2 * L * r, on = N * r;
        const Coef k = in_service(k0, m, (int32_t)l, r);
        const double u = ld(o.x + m.x_vm + on, fb), w = ld(o.x + m.x_vm + on, tb);
        const double th = ld(o.x + m.x_va + on, fb) - ld(o.x + m.x_va + on, tb);
        double S, C;
        sincos(th, &S, &C);
        st(o.g + m.x_p + oa, l, flow1(k.Gff, 0.0, k.Gft, k.Bft, u, w, C, S).F);
        st(o.g + m.x_q + oa, l, flow1(-k.Bff, 0.0, -k.Bft, k.Gft, u, w, C, S).F);
        st(o.g + m.x_p + oa + L, l, flow1(0.0, k.Gtt, k.Gtf, -k.Btf, u, w, C, S).F);
        st(o.g + m.x_q + oa + L, l, flow1(0.0, -k.Btt, -k.Btf, -k.Gtf, u, w, C, S).F);
    }
}

// ================================================================== phase 2
struct Slot {
    int32_t kind, ref, bus, other, jpos, h0, h1, h2;
};
__device__ __forceinline__ Slot load_slot(const DevModel& m, int32_t w) {
    const int4* p = reinterpret_cast<const int4*>(m.slots) + (size_t)w * kBlock * 2;
    const int4 a = ld(p, 2 * threadIdx.x), b = ld(p, 2 * threadIdx.x + 1);
    return Slot{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}

// Output positions in the bus wave: the full slot's fields (one launch) or
// those formed from the compact slot (two launches).
#define H0 (SINGLE ? sl.h0 : h0)
#define H1 (SINGLE ? sl.h1 : h1)
#define H2 (SINGLE ? sl.h2 : h2)
#define JP (SINGLE ? sl.jpos : jp)
// RECT: the rectangular form (bus blocks vr, vi; records [D, Bs, D, A, P, Q];
// a voltage-magnitude row per head).  EXT: the model has storage units or
// devices (lanes of the generator type with kind bit 2 or 4); without them
// the kernel holds none of their code or kernel arguments.
template <bool SINGLE, bool RECT = false, bool EXT = false>
__device__ void wave_task(const DevModel& m, const EvalOut& o, int32_t w, int32_t r, double* lds) {
    const int32_t lane = threadIdx.x;
    const bool wantC = o.c != nullptr, wantH = o.H != nullptr;
    // one launch: a half-edge lane's branch terms depend only on the lane,
    // so they load together with the descriptor
    Coef k{};
    if (SINGLE && wantH) {
        const double2* kc = reinterpret_cast<const double2*>(m.slot_coef) + (size_t)w * kBlock * 4;
        const double2 c01 = ld(kc, 4 * lane), c23 = ld(kc, 4 * lane + 1);
        const double2 c45 = ld(kc, 4 * lane + 2), c67 = ld(kc, 4 * lane + 3);
        k = Coef{c01.x, c01.y, c23.x, c23.y, c45.x, c45.y, c67.x, c67.y};
    }
    // the descriptor: the full slot (one launch, which also needs the
    // neighbour bus), else the compact 8-byte slot, whose output positions
    // come from the head lane's per-bus offsets
    Slot sl;
    int32_t kind, len;
    uint32_t bus, ref;
    if (SINGLE) {
        sl = load_slot(m, w);
        kind = sl.kind;
        len = (kind >> 8) & 0xff;
        bus = (uint32_t)sl.bus;
        ref = (uint32_t)sl.ref;
    } else {
        const int2 c = ld(reinterpret_cast<const int2*>(m.slots_c) + (size_t)w * kBlock, (uint32_t)lane);
        kind = c.x;
        len = ((kind >> 8) & 63) + 1;
        bus = ref = (uint32_t)c.y;
    }
    const int32_t type = kind & 3;
    const uint32_t side = (kind & 4) ? 0u : 1u;  // the half-edge sits at its branch's from bus
    const bool leader = kind & 8;               // len: segment (head) or group (leader) length
    const int64_t N = m.N, G = m.G;
    {  // replica r
        const int64_t on = N * r;
        // every lane type issues its loads before any arithmetic: the lane
        // types of a wave run one after another, and a type that used its
        // loads before the next type's branch would cost the wave one
        // memory round trip per lane type.  The loaded values are read only
        // under their own lane type and get no default: writing a default
        // into a register another type's load is still filling would make
        // the wave wait for that load.
        double gs, bs, vm_i, vr_i, pd, qd, yp, yq, ymag, gp, gq;
        double2 ra, rb, rc;
        HeIn e;
        RHeIn re;
        int32_t jrow, hva0, hvm0, nlo, nd;  // the head's per-bus offsets (compact slots)
        if (type == SK_HEAD) {
            gs = ld(m.gs, bus);
            bs = ld(m.bs, bus);
            vm_i = ld(o.x + m.x_vm + on, bus);  // rectangular: vi_i
            if (RECT) {
                vr_i = ld(o.x + m.x_va + on, bus);
                if (wantH) ymag = ld(o.y + m.c_vmag + on, bus);
            }
            if (!SINGLE) {
                if (o.J) jrow = ld(m.jbal_off, bus);
                if (wantH) {
                    hva0 = ld(m.hva_off, bus);
                    hvm0 = ld(m.hvm_off, bus);
                    nlo = ld(m.nlo, bus);
                    nd = ld(m.ndist, bus);
                }
            }
            if (wantC) {
                const int64_t ol = (int64_t)m.load_stride * r;
                pd = ld(m.pd + ol, bus);
                qd = ld(m.qd + ol, bus);
            }
            if (wantH) {
                yp = ld(o.y + m.c_balp + on, bus);
                yq = ld(o.y + m.c_balq + on, bus);
            }
        } else if (type == SK_EDGE && SINGLE) {
            const uint32_t other = (uint32_t)sl.other;
            if (RECT)
                rect_edge_load(m, o, ref, side, side ? other : bus, side ? bus : other, r, re);
            else
                half_edge_load(m, o, ref, side, side ? other : bus, side ? bus : other, r, e);
        } else if (type == SK_EDGE) {
            const double2* rec = reinterpret_cast<const double2*>(rec_side(m, r, (int32_t)side));
            if (wantH) {
                const uint32_t q = (kRecStride / 2) * ref;
                ra = ld(rec, q);
                rb = ld(rec, q + 1);
                if (wantC) rc = ld(rec, q + 2);
            } else if (wantC) {  // compact records [P, Q]
                rc = ld(rec, ref);
            }
        } else if (EXT && type == SK_GEN && (kind & 4)) {
            // a storage unit: ps, qs (and for its (vm, vm) term the loss
            // rows' multipliers and r, x), held in the generator / head
            // registers (gp, gq, yp, yq, gs, bs), which a lane of another
            // type does not use
            const int64_t S = m.S;
            if (wantC || wantH) {
                gp = ld(o.x + m.x_ps + S * r, ref);
                gq = ld(o.x + m.x_qs + S * r, ref);
            }
            if (wantH) {
                yp = ld(o.y + m.c_slp + S * r, ref);
                yq = ld(o.y + m.c_slq + S * r, ref);
                gs = ld(m.stor_par + SP_R * S, ref);
                bs = ld(m.stor_par + SP_X * S, ref);
            }
        } else if (EXT && type == SK_GEN && (kind & 16)) {
            // a device: u and its balance coefficients cp, cq
            const int64_t D = m.D;
            if (wantC) gp = ld(o.x + m.x_u + D * r, ref);
            if (wantC || o.J) {
                gs = ld(m.dev_par + DP_CP * D, ref);
                bs = ld(m.dev_par + DP_CQ * D, ref);
            }
        } else if (type == SK_GEN && wantC) {
            gp = ld(o.x + m.x_pg + G * (m.npg > 1 ? r : 0), ref);
            gq = ld(o.x + m.x_qg + G * r, ref);
        }
        // a storage lane's (vm, vm) term needs its bus's vm: the head's
        double vm_h = 0.0;
        if (EXT && wantH && m.S > 0) vm_h = __shfl(vm_i, SINGLE ? (sl.other & 63) : ((kind >> 14) & 63), kBlock);
        double v[kRec] = {0, 0, 0, 0, 0, 0};
        double base_p = 0.0, base_q = 0.0, shunt = 0.0;
        if (type == SK_HEAD) {
            // vm^2 (rectangular: vr^2 + vi^2)
            const double v2 = RECT ? vr_i * vr_i + vm_i * vm_i : vm_i * vm_i;
            if (wantC) {
                base_p = pd + gs * v2;
                base_q = qd - bs * v2;
            }
            if (wantH) shunt = 2.0 * gs * yp - 2.0 * bs * yq + (RECT ? 2.0 * ymag : 0.0);
        } else if (type == SK_EDGE && SINGLE) {
            if (RECT)
                rect_edge_record(m, o, re, ref, side, k, r, v);
            else
                half_edge_record(m, o, e, ref, side, k, r, v);
        } else if (type == SK_EDGE) {
            if (wantH) {
                v[R_TT] = ra.x;
                v[R_MA] = ra.y;
                v[R_MM] = rb.x;
                v[R_UW] = rb.y;
            }
            if (wantC) {
                v[R_P] = rc.x;
                v[R_Q] = rc.y;
            }
        } else if (EXT && type == SK_GEN && (kind & 4)) {  // storage: +ps, +qs
            if (wantC) {
                v[R_P] = gp;
                v[R_Q] = gq;
            }
            if (wantH) v[R_MM] = stor_vmvm(gp, gq, vm_h, yp, yq, gs, bs);
        } else if (EXT && type == SK_GEN && (kind & 16)) {  // device: +cp u, +cq u
            if (wantC) {
                v[R_P] = gs * gp;
                v[R_Q] = bs * gp;
            }
        } else if (type == SK_GEN && wantC) {
            v[R_P] = -gp;
            v[R_Q] = -gq;
        }
        // output positions: balance Jacobian entry, Hessian entries of the
        // bus (-1: absent).  With compact slots every lane joins the
        // shuffles; only heads and leaders use the Hessian positions.  They
        // are formed here, once all loads have landed, so that the offsets
        // are not live through the reductions below.
        // (The full slot holds them; it is read at the stores.)
        int32_t jp = 0, h0, h1, h2;
        if constexpr (!SINGLE) {
            const int32_t hl = (kind >> 14) & 63;
            // the rectangular balance rows lead with two bus entries
            if (o.J) jp = __shfl(jrow, hl, kBlock) + ((kind >> 20) & 63) + (RECT && type != SK_HEAD ? 1 : 0);
            if (wantH && RECT) {
                const int32_t hva_b = __shfl(hva0, hl, kBlock), hvm_b = __shfl(hvm0, hl, kBlock);
                const int32_t nd_b = __shfl(nd, hl, kBlock);
                if (type == SK_HEAD) {  // (vr_i, vr_i), (vi_i, vi_i)
                    h0 = hva_b + nlo;
                    h1 = -1;
                    h2 = hvm_b + nd_b + nlo;
                } else {  // (vr_i, vr_k), (vi_i, vr_k), (vi_i, vi_k) of the group
                    const int32_t grp = (int32_t)((uint32_t)kind >> 26);
                    const bool klo = kind & 16;
                    h0 = klo ? hva_b + grp : -1;
                    h1 = hvm_b + grp;
                    h2 = klo ? hvm_b + nd_b + grp : -1;
                }
            } else if (wantH) {
                const int32_t hva_b = __shfl(hva0, hl, kBlock), hvm_b = __shfl(hvm0, hl, kBlock);
                const int32_t nd_b = __shfl(nd, hl, kBlock);
                if (type == SK_HEAD) {  // (va_i, va_i), (vm_i, va_i), (vm_i, vm_i)
                    const bool nodeg = kind & 64;
                    h0 = nodeg ? -1 : hva_b + nlo;
                    h1 = nodeg ? -1 : hvm_b + nlo;
                    h2 = nodeg ? hvm_b : hvm_b + nd_b + 1 + nlo;
                } else {  // (va_i, va_k), (vm_i, va_k), (vm_i, vm_k) of the group
                    const int32_t grp = (int32_t)((uint32_t)kind >> 26);
                    const bool klo = kind & 16, khi = kind & 32;
                    h0 = klo ? hva_b + grp : -1;
                    h1 = hvm_b + grp + (khi ? 1 : 0);
                    h2 = klo ? hvm_b + nd_b + 1 + grp : -1;
                }
            }
        }
        if (wantC || wantH) {
            for (int q = 0; q < kRec; q++) lds[q * kBlock + lane] = v[q];
            __syncthreads();
            if (type == SK_HEAD) {
                double sp = base_p, sq = base_q, daa = 0.0, dma = 0.0, dmm = 0.0;
                auto add = [&](int32_t j) {  // the segment, in order
                    sp += lds[R_P * kBlock + lane + j];
                    sq += lds[R_Q * kBlock + lane + j];
                    daa += lds[R_TT * kBlock + lane + j];
                    dma += lds[R_MA * kBlock + lane + j];
                    dmm += lds[R_MM * kBlock + lane + j];
                };
                if constexpr (SINGLE) {
                    for (int32_t j = 1; j < len; j++) add(j);
                } else {
#pragma unroll 4  // the compiler's deeper unrolling spills in the two-launch bus kernel
                    for (int32_t j = 1; j < len; j++) add(j);
                }
                if (wantC) {
                    st(o.c + m.c_balp + on, bus, sp);
                    st(o.c + m.c_balq + on, bus, sq);
                    if (RECT) st(o.c + m.c_vmag + on, bus, vr_i * vr_i + vm_i * vm_i);
                }
                // The Hessian entries of a bus are single scattered values;
                // in the two-launch shape they merge into whole lines in L2
                // before they are written back (streaming them: 16-point
                // batch 55 -> 60 us, 64-scenario batch 114 -> 128 us), while
                // in the one launch streaming them is faster.
                if (wantH && RECT) {  // the two diagonals; no (vi_i, vr_i) entry
                    double* hva = o.H + m.h_va + m.hva_rep * r;
                    double* hvm = o.H + m.h_vm + m.hvm_rep * r;
                    st_sel<SINGLE>(hva, (uint32_t)H0, daa + shunt);
                    st_sel<SINGLE>(hvm, (uint32_t)H2, dmm + shunt);
                } else if (wantH) {
                    double* hva = o.H + m.h_va + m.hva_rep * r;
                    double* hvm = o.H + m.h_vm + m.hvm_rep * r;
                    if (H0 >= 0) st_sel<SINGLE>(hva, (uint32_t)H0, daa);
                    if (H1 >= 0) st_sel<SINGLE>(hvm, (uint32_t)H1, dma);
                    st_sel<SINGLE>(hvm, (uint32_t)H2, dmm + shunt);
                }
            } else if (type == SK_EDGE && wantH && leader) {
                // the neighbour group (parallel branches to one bus), in order
                double tt = v[R_TT], ma = v[R_MA], uw = v[R_UW];
                for (int32_t j = 1; j < len; j++) {
                    tt += lds[R_TT * kBlock + lane + j];
                    ma += lds[R_MA * kBlock + lane + j];
                    uw += lds[R_UW * kBlock + lane + j];
                }
                double* hva = o.H + m.h_va + m.hva_rep * r;
                double* hvm = o.H + m.h_vm + m.hvm_rep * r;
                // polar: (va_i, va_k) = -TT, (vm_i, va_k) = -MA, (vm_i, vm_k) = UW;
                // rectangular: (vr_i, vr_k) = A, (vi_i, vr_k) = Bs, (vi_i, vi_k) = A
                if (H0 >= 0) st_sel<SINGLE>(hva, (uint32_t)H0, RECT ? uw : -tt);
                st_sel<SINGLE>(hvm, (uint32_t)H1, RECT ? ma : -ma);
                if (H2 >= 0) st_sel<SINGLE>(hvm, (uint32_t)H2, uw);
            }
            __syncthreads();  // LDS is reused by the next replica
        }
        if (o.J && type != SK_IDLE) {
            double vp, vq;
            if (type == SK_HEAD) {
                vp = 2.0 * gs * vm_i;
                vq = -2.0 * bs * vm_i;
            } else if (EXT && type == SK_GEN && (kind & 16)) {  // device: cp, cq
                vp = gs;
                vq = bs;
            } else {  // arcs and storage units +1, generators -1
                vp = vq = (type == SK_EDGE || (EXT && (kind & 4))) ? 1.0 : -1.0;
            }
            if (RECT && type == SK_HEAD) {
                // (vr_i, vi_i) of both balance rows, then the magnitude row
                st(o.J + m.j_balp + m.jbal_rep * r, (uint32_t)JP, 2.0 * gs * vr_i);
                st(o.J + m.j_balq + m.jbal_rep * r, (uint32_t)JP, -2.0 * bs * vr_i);
                st(o.J + m.j_balp + m.jbal_rep * r, (uint32_t)JP + 1, vp);
                st(o.J + m.j_balq + m.jbal_rep * r, (uint32_t)JP + 1, vq);
                st(o.J + m.j_vmag + 2 * on, 2 * bus, 2.0 * vr_i);
                st(o.J + m.j_vmag + 2 * on, 2 * bus + 1, 2.0 * vm_i);
            } else {
                st(o.J + m.j_balp + m.jbal_rep * r, (uint32_t)JP, vp);
                st(o.J + m.j_balq + m.jbal_rep * r, (uint32_t)JP, vq);
            }
        }
        if (o.g && type == SK_HEAD) {
            st(o.g + m.x_va + on, bus, 0.0);
            st(o.g + m.x_vm + on, bus, 0.0);
        }
    }
}
#undef H0
#undef H1
#undef H2
#undef JP

// J^T v, phase 2: va / vm (rectangular: vr / vi) entries of the packed buses.
template <bool RECT = false, bool EXT = false>
__device__ void jt_wave_task(const DevModel& m, const EvalOut& o, int32_t w, int32_t r, double* lds) {
    const int32_t lane = threadIdx.x;
    // the compact slot: lane type, side, segment length; the index is the
    // bus (head) or the branch (half-edge)
    const int2 sc = ld(reinterpret_cast<const int2*>(m.slots_c) + (size_t)w * kBlock, (uint32_t)lane);
    const int32_t type = sc.x & 3;
    const uint32_t side = (sc.x & 4) ? 0u : 1u;
    const int32_t len = ((sc.x >> 8) & 63) + 1;
    const int64_t N = m.N;
    const uint32_t bus = (uint32_t)sc.y, ref = (uint32_t)sc.y;
    const double* x = o.x;
    const double* v = o.y;
    {  // replica r
        const int64_t on = N * r;
        // the head lanes' loads go out with the half-edge lanes' records
        // (one memory round trip); loaded values get no default (see
        // wave_task)
        double2 t;
        double vm, vr, gs, bs, vp, vq, vg;
        int32_t q0, q1;
        if (type == SK_EDGE) {
            t = ld(reinterpret_cast<const double2*>(jt_rec_side(m, r, (int32_t)side)), ref);
        } else if (EXT && type == SK_GEN && (sc.x & 4)) {
            // a storage unit's loss rows: ps, qs, their multipliers, r, x
            // (in the registers of the head's loads)
            const int64_t S = m.S;
            vr = ld(x + m.x_ps + S * r, ref);
            vg = ld(x + m.x_qs + S * r, ref);
            vp = ld(v + m.c_slp + S * r, ref);
            vq = ld(v + m.c_slq + S * r, ref);
            gs = ld(m.stor_par + SP_R * S, ref);
            bs = ld(m.stor_par + SP_X * S, ref);
        } else if (type == SK_HEAD) {
            vm = ld(x + m.x_vm + on, bus);  // rectangular: vi
            if (RECT) {
                vr = ld(x + m.x_va + on, bus);
                vg = ld(v + m.c_vmag + on, bus);
            }
            gs = ld(m.gs, bus);
            bs = ld(m.bs, bus);
            vp = ld(v + m.c_balp + on, bus);
            vq = ld(v + m.c_balq + on, bus);
            q0 = ld(m.ref_ptr, bus);
            q1 = ld(m.ref_ptr, bus + 1);
        }
        double vm_h = 0.0;
        if (EXT && m.S > 0) vm_h = __shfl(vm, (sc.x >> 14) & 63, kBlock);
        const bool stor = EXT && type == SK_GEN && (sc.x & 4);
        lds[0 * kBlock + lane] = type == SK_EDGE ? t.x : 0.0;
        lds[1 * kBlock + lane] = type == SK_EDGE ? t.y : stor ? jt_stor_vm(vr, vg, vm_h, vp, vq, gs, bs) : 0.0;
        __syncthreads();
        if (type == SK_HEAD) {
            double sa = 0.0, sm = 0.0;
            for (int32_t j = 1; j < len; j++) {
                sa += lds[0 * kBlock + lane + j];
                sm += lds[1 * kBlock + lane + j];
            }
            double sref = 0.0;
            for (int32_t q = q0; q < q1; q++)  // the reference row (one bus)
                sref += ld(v + m.c_ref + (int64_t)m.R * r, (uint32_t)ld(m.ref_list, (uint32_t)q));
            if (RECT) {  // balance rows' shunt terms and the magnitude row; ref row on vi
                sa += 2.0 * gs * vr * vp - 2.0 * bs * vr * vq + 2.0 * vr * vg;
                sm += 2.0 * gs * vm * vp - 2.0 * bs * vm * vq + 2.0 * vm * vg + sref;
            } else {
                sa += sref;
                sm += 2.0 * gs * vm * vp - 2.0 * bs * vm * vq;
            }
            st(o.g + m.x_va + on, bus, sa);
            st(o.g + m.x_vm + on, bus, sm);
        }
        __syncthreads();
    }
}

// The record of half-edge `code` (branch << 1 | from-side flag) of a big
// bus: recomputed in a single launch, else read from the branch phase.
template <bool SINGLE, bool RECT>
__device__ __forceinline__ void big_record(const DevModel& m, const EvalOut& o, int32_t code, int32_t r,
                                           const double* rec0, const double* rec1, double (&v)[kRec]) {
    const uint32_t l = (uint32_t)(code >> 1), side = (code & 1) ? 0u : 1u;
    if (SINGLE) {
        for (int q = 0; q < kRec; q++) v[q] = 0.0;
        const Coef k = o.H ? load_coef(m, l) : Coef{};
        if (RECT) {
            RHeIn e{};
            rect_edge_load(m, o, l, side, (uint32_t)ld(m.f_bus, l), (uint32_t)ld(m.t_bus, l), r, e);
            rect_edge_record(m, o, e, l, side, k, r, v);
        } else {
            HeIn e{};
            half_edge_load(m, o, l, side, (uint32_t)ld(m.f_bus, l), (uint32_t)ld(m.t_bus, l), r, e);
            half_edge_record(m, o, e, l, side, k, r, v);
        }
    } else if (o.H) {
        const double* rec = (side == 0 ? rec0 : rec1) + (int64_t)l * kRecStride;
        for (int q = 0; q < kRec; q++) v[q] = rec[q];
    } else {  // compact records [P, Q]
        const double* rec = (side == 0 ? rec0 : rec1) + (int64_t)l * kRecPQ;
        for (int q = 0; q < kRec; q++) v[q] = 0.0;
        v[R_P] = rec[0];
        v[R_Q] = rec[1];
    }
}

// A bus whose segment does not fit a wave: the workgroup sums its
// half-edges' records (lane-strided, then a fixed wave tree).
template <bool SINGLE, bool RECT = false, bool EXT = false>
__device__ void big_task(const DevModel& m, const EvalOut& o, int32_t idx, int32_t r) {
    const int32_t b = m.big_bus[idx];
    const int32_t e0 = m.adj_ptr[b], e1 = m.adj_ptr[b + 1], deg = e1 - e0;
    const int64_t N = m.N, G = m.G;
    const double* x = o.x;
    const bool wantH = o.H != nullptr, wantC = o.c != nullptr;
    const int32_t g0 = m.gen_ptr[b], ng = m.gen_ptr[b + 1] - g0;
    const double gs = m.gs[b], bs = m.bs[b];
    {  // replica r
        const int64_t bi = b + N * r;
        const double vm = x[m.x_vm + bi];             // rectangular: vi
        const double vr = RECT ? x[m.x_va + bi] : 0.0;
        const double v2 = RECT ? vr * vr + vm * vm : vm * vm;
        const double* rec0 = rec_side(m, r, 0);
        const double* rec1 = rec_side(m, r, 1);
        if (wantC || wantH) {
            double sp = 0.0, sq = 0.0, daa = 0.0, dma = 0.0, dmm = 0.0;
            for (int32_t q = threadIdx.x; q < deg; q += kBlock) {
                double rec[kRec];
                big_record<SINGLE, RECT>(m, o, m.he[e0 + q], r, rec0, rec1, rec);
                if (wantC) {
                    sp += rec[R_P];
                    sq += rec[R_Q];
                }
                if (wantH) {
                    daa += rec[R_TT];
                    dma += rec[R_MA];
                    dmm += rec[R_MM];
                }
            }
            sp = wave_sum(sp);
            sq = wave_sum(sq);
            daa = wave_sum(daa);
            dma = wave_sum(dma);
            dmm = wave_sum(dmm);
            if (wantH) {  // each neighbour group's first half-edge sums the group
                const int64_t hva = m.h_va + m.hva_rep * r + m.hva_off[b];
                const int64_t hvm = m.h_vm + m.hvm_rep * r + m.hvm_off[b];
                for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += kBlock) {
                    const int32_t grp = m.he_grp[e];
                    if (e > e0 && m.he_grp[e - 1] == grp) continue;
                    const int32_t code = m.he[e], l = code >> 1;
                    const int32_t k = (code & 1) ? m.t_bus[l] : m.f_bus[l];
                    double tt = 0.0, ma = 0.0, uw = 0.0;
                    for (int32_t q = e; q < e1 && m.he_grp[q] == grp; q++) {
                        double rec[kRec];
                        big_record<SINGLE, RECT>(m, o, m.he[q], r, rec0, rec1, rec);
                        tt += rec[R_TT];
                        ma += rec[R_MA];
                        uw += rec[R_UW];
                    }
                    if (RECT) {  // (vr_i, vr_k) = A, (vi_i, vr_k) = Bs, (vi_i, vi_k) = A
                        o.H[hvm + grp] = ma;
                        if (k < b) {
                            o.H[hva + grp] = uw;
                            o.H[hvm + m.ndist[b] + grp] = uw;
                        }
                    } else if (k < b) {
                        o.H[hva + grp] = -tt;
                        o.H[hvm + grp] = -ma;
                        o.H[hvm + m.ndist[b] + 1 + grp] = uw;
                    } else {
                        o.H[hvm + grp + 1] = -ma;
                    }
                }
            }
            if (threadIdx.x == 0) {
                if (wantC) {
                    const int64_t ld_ = b + (int64_t)m.load_stride * r;
                    double cp = m.pd[ld_] + gs * v2 + sp, cq = m.qd[ld_] - bs * v2 + sq;
                    const int64_t pgb = m.x_pg + G * (m.npg > 1 ? r : 0), qgb = m.x_qg + G * r;
                    for (int32_t q = 0; q < ng; q++) {
                        cp -= x[pgb + m.gen_list[g0 + q]];
                        cq -= x[qgb + m.gen_list[g0 + q]];
                    }
                    for (int32_t q = EXT ? m.st_ptr[b] : 0; q < (EXT ? m.st_ptr[b + 1] : 0); q++) {  // storage
                        const int64_t e = m.st_list[q] + (int64_t)m.S * r;
                        cp += x[m.x_ps + e];
                        cq += x[m.x_qs + e];
                    }
                    for (int32_t q = EXT ? m.dv_ptr[b] : 0; q < (EXT ? m.dv_ptr[b + 1] : 0); q++) {  // devices
                        const int32_t d = m.dv_list[q];
                        const double u = x[m.x_u + d + (int64_t)m.D * r];
                        cp += m.dev_par[DP_CP * (int64_t)m.D + d] * u;
                        cq += m.dev_par[DP_CQ * (int64_t)m.D + d] * u;
                    }
                    o.c[m.c_balp + bi] = cp;
                    o.c[m.c_balq + bi] = cq;
                    if (RECT) o.c[m.c_vmag + bi] = v2;
                }
                if (wantH) {
                    double shunt = 2.0 * gs * o.y[m.c_balp + bi] - 2.0 * bs * o.y[m.c_balq + bi] +
                                   (RECT ? 2.0 * o.y[m.c_vmag + bi] : 0.0);
                    for (int32_t q = EXT ? m.st_ptr[b] : 0; q < (EXT ? m.st_ptr[b + 1] : 0); q++) {  // storage (vm, vm)
                        const int32_t u = m.st_list[q];
                        const int64_t e = u + (int64_t)m.S * r;
                        shunt += stor_vmvm(x[m.x_ps + e], x[m.x_qs + e], vm, o.y[m.c_slp + e], o.y[m.c_slq + e],
                                           m.stor_par[SP_R * (int64_t)m.S + u], m.stor_par[SP_X * (int64_t)m.S + u]);
                    }
                    const int64_t hva = m.h_va + m.hva_rep * r + m.hva_off[b];
                    const int64_t hvm = m.h_vm + m.hvm_rep * r + m.hvm_off[b];
                    const int32_t nlo = m.nlo[b];
                    if (RECT) {
                        o.H[hva + nlo] = daa + shunt;
                        o.H[hvm + m.ndist[b] + nlo] = dmm + shunt;
                    } else {
                        o.H[hva + nlo] = daa;
                        o.H[hvm + nlo] = dma;
                        o.H[hvm + m.ndist[b] + 1 + nlo] = dmm + shunt;
                    }
                }
            }
        }
        if (o.J) {
            double* Jp = o.J + m.j_balp + m.jbal_rep * r + m.jbal_off[b];
            double* Jq = o.J + m.j_balq + m.jbal_rep * r + m.jbal_off[b];
            if (RECT) {  // (vr_i, vi_i), generators, arcs; then the magnitude row
                for (int32_t q = threadIdx.x; q < 2 + ng + deg; q += kBlock) {
                    Jp[q] = q == 0 ? 2.0 * gs * vr : q == 1 ? 2.0 * gs * vm : (q <= ng + 1 ? -1.0 : 1.0);
                    Jq[q] = q == 0 ? -2.0 * bs * vr : q == 1 ? -2.0 * bs * vm : (q <= ng + 1 ? -1.0 : 1.0);
                }
                if (threadIdx.x == 0) {
                    o.J[m.j_vmag + 2 * bi] = 2.0 * vr;
                    o.J[m.j_vmag + 2 * bi + 1] = 2.0 * vm;
                }
            } else {
                for (int32_t q = threadIdx.x; q < 1 + ng + deg; q += kBlock) {
                    Jp[q] = q == 0 ? 2.0 * gs * vm : (q <= ng ? -1.0 : 1.0);
                    Jq[q] = q == 0 ? -2.0 * bs * vm : (q <= ng ? -1.0 : 1.0);
                }
            }
            // storage units (+1) and devices (cp, cq) follow the arcs
            const int32_t nbv = RECT ? 2 : 1, ns = EXT ? m.st_ptr[b + 1] - m.st_ptr[b] : 0;
            const int32_t nd = EXT ? m.dv_ptr[b + 1] - m.dv_ptr[b] : 0, q0 = nbv + ng + deg;
            for (int32_t q = threadIdx.x; q < ns + nd; q += kBlock) {
                double vp = 1.0, vq = 1.0;
                if (q >= ns) {
                    const int32_t d = m.dv_list[m.dv_ptr[b] + q - ns];
                    vp = m.dev_par[DP_CP * (int64_t)m.D + d];
                    vq = m.dev_par[DP_CQ * (int64_t)m.D + d];
                }
                Jp[q0 + q] = vp;
                Jq[q0 + q] = vq;
            }
        }
        if (o.g && threadIdx.x == 0) {
            o.g[m.x_va + bi] = 0.0;
            o.g[m.x_vm + bi] = 0.0;
        }
    }
}

template <bool RECT = false, bool EXT = false>
__device__ void jt_big_task(const DevModel& m, const EvalOut& o, int32_t idx, int32_t r) {
    const int32_t b = m.big_bus[idx];
    const int32_t e0 = m.adj_ptr[b], deg = m.adj_ptr[b + 1] - e0;
    const int64_t N = m.N;
    const double* x = o.x;
    const double* v = o.y;
    {  // replica r
        const double* rec0 = jt_rec_side(m, r, 0);
        const double* rec1 = jt_rec_side(m, r, 1);
        double sa = 0.0, sm = 0.0;
        for (int32_t q = threadIdx.x; q < deg; q += kBlock) {
            const int32_t code = m.he[e0 + q];
            const double* rec = ((code & 1) ? rec0 : rec1) + (int64_t)(code >> 1) * 2;
            sa += rec[0];
            sm += rec[1];
        }
        sa = wave_sum(sa);
        sm = wave_sum(sm);
        if (threadIdx.x == 0) {
            const int64_t bi = b + N * r;
            double sref = 0.0;
            for (int32_t q = m.ref_ptr[b]; q < m.ref_ptr[b + 1]; q++)
                sref += v[m.c_ref + m.ref_list[q] + (int64_t)m.R * r];
            const double vm = x[m.x_vm + bi];  // rectangular: vi
            const double vp = v[m.c_balp + bi], vq = v[m.c_balq + bi];
            if (RECT) {
                const double vr = x[m.x_va + bi], vg = v[m.c_vmag + bi];
                sa += 2.0 * m.gs[b] * vr * vp - 2.0 * m.bs[b] * vr * vq + 2.0 * vr * vg;
                sm += 2.0 * m.gs[b] * vm * vp - 2.0 * m.bs[b] * vm * vq + 2.0 * vm * vg + sref;
            } else {
                sa += sref;
                sm += 2.0 * m.gs[b] * vm * vp - 2.0 * m.bs[b] * vm * vq;
                for (int32_t q = EXT ? m.st_ptr[b] : 0; q < (EXT ? m.st_ptr[b + 1] : 0); q++) {  // storage
                    const int32_t u = m.st_list[q];
                    const int64_t e = u + (int64_t)m.S * r;
                    sm += jt_stor_vm(x[m.x_ps + e], x[m.x_qs + e], vm, v[m.c_slp + e], v[m.c_slq + e],
                                     m.stor_par[SP_R * (int64_t)m.S + u], m.stor_par[SP_X * (int64_t)m.S + u]);
                }
            }
            o.g[m.x_va + bi] = sa;
            o.g[m.x_vm + bi] = sm;
        }
    }
}

// One objective partial: the wave's terms summed in a fixed tree into
// slot `slot` (generator chunks first, then device chunks; obj_slots).  Two
// launches: a plain store, summed by the objective item after the launch
// boundary.  One launch: the chunk whose arrival completes a self-resetting
// ticket sums every partial in index order.  Partials and ticket are
// device-coherent atomics; the ticket moves only after this wave's partial
// store has completed (s_waitcnt 0).  An acquire-release ticket would also
// write back and invalidate the whole XCD L2 for every chunk, which cost
// 1.6 us of the 10k-bus set.
template <bool SINGLE, bool EXT>
__device__ __forceinline__ void obj_partial(const DevModel& m, const EvalOut& o, int64_t slot, double fk) {
    const double s = wave_sum(fk);
    if (!SINGLE) {
        if (threadIdx.x == 0) m.obj_part[slot] = s;
        return;
    }
    __shared__ int32_t last;
    const int32_t total = EXT ? obj_slots(m) : m.ngchunks * m.npg;
    if (threadIdx.x == 0) {
        __hip_atomic_store(&m.obj_part[slot], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int32_t old = __hip_atomic_fetch_add(m.obj_ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = (old + 1 == total) ? 1 : 0;
    }
    __syncthreads();
    if (last) {
        // acquire at agent scope, once per launch (the last chunk only): the
        // partials below are read after every other chunk's ticket
        // increment, which each issued only once its own partial store had
        // completed
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        double acc = 0.0;
        for (int32_t q = threadIdx.x; q < total; q += kBlock)
            acc += __hip_atomic_load(&m.obj_part[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        acc = wave_sum(acc);
        if (threadIdx.x == 0) {
            *o.f = acc;
            __hip_atomic_store(m.obj_ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------------ generators
// Phase 1: per generator chunk the gradient, the pg Hessian diagonal, the
// reference and ramp rows, and one objective partial per replica (a fixed
// wave tree over the chunk), written with a plain store: the objective item
// of phase 2 reads the partials after the launch boundary.
template <bool SINGLE, bool RECT = false, bool EXT = false>
__device__ void gen_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const uint32_t k = (uint32_t)(chunk * kBlock) + threadIdx.x;
    const double* x = o.x;
    const int64_t G = m.G;
    const bool isgen = k < (uint32_t)m.G, isref = k < (uint32_t)m.R;
    double c2 = 0.0, c1 = 0.0, c0 = 0.0;
    if (isgen) {
        c2 = ld(m.c2, k);
        c1 = ld(m.c1, k);
        c0 = ld(m.c0, k);
    }
    const uint32_t rbus = isref ? (uint32_t)ld(m.ref_bus, k) : 0u;
    {  // replica r; every load before the first store (one in-order completion counter)
        const bool ramp = isgen && m.T > 1 && r >= 1;
        const double pg = (isgen && r < m.npg) ? ld(x + m.x_pg + G * r, k) : 0.0;
        const double pr = ramp ? ld(x + m.x_pg + G * r, k) - ld(x + m.x_pg + G * (r - 1), k) : 0.0;
        // the reference row: va_r (rectangular: vi_r)
        const double var = (isref && o.c) ? ld(x + (RECT ? m.x_vm : m.x_va) + (int64_t)m.N * r, rbus) : 0.0;
        double fk = 0.0;
        if (isgen) {
            if (r < m.npg) {
                fk = c2 * pg * pg + c1 * pg + c0;
                if (o.g) st(o.g + m.x_pg + G * r, k, 2.0 * c2 * pg + c1);
                if (o.H) st(o.H + m.h_pg + G * r, k, 2.0 * o.sigma * c2);
            }
            if (o.g) st(o.g + m.x_qg + G * r, k, 0.0);
            if (ramp) {
                const int64_t row0 = G * (r - 1);
                if (o.c) st(o.c + m.c_ramp + row0, k, pr);
                if (o.J) {
                    st(o.J + m.j_ramp + 2 * row0, 2 * k, -1.0);
                    st(o.J + m.j_ramp + 2 * row0, 2 * k + 1, 1.0);
                }
            }
        }
        if (isref) {
            const int64_t row0 = (int64_t)m.R * r;
            if (o.c) st(o.c + m.c_ref + row0, k, var);
            if (o.J) st(o.J + m.j_ref + row0, k, 1.0);
        }
        if (o.f && r < m.npg) obj_partial<SINGLE, EXT>(m, o, chunk + (int64_t)m.ngchunks * r, fk);
    }
}

// Phase 2 of a two-launch model: f = the partials summed lane-strided in
// index order, then a fixed wave tree.
template <bool EXT>
__device__ void obj_task(const DevModel& m, const EvalOut& o) {
    if (o.f == nullptr) return;
    const int32_t total = EXT ? obj_slots(m) : m.ngchunks * m.npg;
    double acc = 0.0;
    for (int32_t q = threadIdx.x; q < total; q += kBlock) acc += m.obj_part[q];
    acc = wave_sum(acc);
    if (threadIdx.x == 0) *o.f = acc;
}

__device__ void jt_gen_task(const DevModel& m, const EvalOut& o, int32_t idx, int32_t r) {
    const int64_t G = m.G, N = m.N;
    const double* v = o.y;
    if (m.npg == 1 && m.nrep > 1) {
        // pg shared by every contingency copy: one wave per generator, lanes
        // over the copies, then a fixed-order wave sum
        const int32_t k = idx;
        const int32_t bus = m.gen_bus[k];
        double acc = 0.0;
        for (int32_t s = threadIdx.x; s < m.nrep; s += kBlock) {
            acc -= v[m.c_balp + bus + N * s];
            o.g[m.x_qg + k + G * s] = -v[m.c_balq + bus + N * s];
        }
        acc = wave_sum(acc);
        if (threadIdx.x == 0) o.g[m.x_pg + k] = acc;
        return;
    }
    const uint32_t k = (uint32_t)(idx * kBlock) + threadIdx.x;
    if (k >= (uint32_t)m.G) return;
    const uint32_t bus = (uint32_t)ld(m.gen_bus, k);
    {  // replica r; both loads before the stores
        const double yq = ld(v + m.c_balq + N * r, bus);
        double acc = -ld(v + m.c_balp + N * r, bus);
        if (m.T > 1) {
            if (r >= 1) acc += ld(v + m.c_ramp + G * (r - 1), k);
            if (r + 1 < m.T) acc -= ld(v + m.c_ramp + G * r, k);
        }
        st(o.g + m.x_qg + G * r, k, -yq);
        st(o.g + m.x_pg + G * r, k, acc);
    }
}

// ----------------------------------------------------- storage and devices
// Storage units (the storage model of Geth, Coffrin and Fobes 2020 that the
// paper cites, Sec. III-C3), one lane per unit and replica (period).  With
// S2 = ps^2 + qs^2 and the squared converter current i2 = S2 / vm^2:
//   soc     se - se_prev - dt (eta_c sc - sd / eta_d)     (se_prev = e0 at t = 0)
//   loss_p  ps + sd - sc - ploss - r i2
//   loss_q  qs - qsc - qloss - x i2
//   thermal S2 - rating^2;  comp  sc sd
// The unit's own rows, their Jacobian entries, its Hessian rows (ps, qs,
// sd) and the zero gradient of its variables are written here; its
// balance-row entries and its (vm, vm) Hessian term belong to its bus's
// segment (a storage lane there).
__device__ void stor_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const uint32_t u = (uint32_t)(chunk * kBlock) + threadIdx.x;
    if (u >= (uint32_t)m.S) return;
    const int64_t S = m.S, so = S * r;
    const double* P = m.stor_par;
    const double* x = o.x;
    // every load before the first store
    const uint32_t bus = (uint32_t)ld(m.stor_bus, u);
    const double ps = ld(x + m.x_ps + so, u), qs = ld(x + m.x_qs + so, u);
    const double qsc = ld(x + m.x_qsc + so, u), se = ld(x + m.x_se + so, u);
    const double sc = ld(x + m.x_sc + so, u), sd = ld(x + m.x_sd + so, u);
    const double se0 = r >= 1 ? ld(x + m.x_se + so - S, u) : ld(P + SP_E0 * S, u);
    const double vm = ld(x + m.x_vm + (int64_t)m.N * r, bus);
    const double etac = ld(P + SP_ETAC * S, u), etad = ld(P + SP_ETAD * S, u);
    const double rr = ld(P + SP_R * S, u), xx = ld(P + SP_X * S, u);
    const double pls = ld(P + SP_PLOSS * S, u), qls = ld(P + SP_QLOSS * S, u), rat = ld(P + SP_RATING * S, u);
    double ylp = 0.0, ylq = 0.0, yth = 0.0, ycm = 0.0;
    if (o.H) {
        ylp = ld(o.y + m.c_slp + so, u);
        ylq = ld(o.y + m.c_slq + so, u);
        yth = ld(o.y + m.c_sth + so, u);
        if (m.comp) ycm = ld(o.y + m.c_scmp + so, u);
    }
    const double dt = m.stor_dt;
    const double iv2 = 1.0 / (vm * vm), iv3 = iv2 / vm;
    const double S2 = ps * ps + qs * qs, i2 = S2 * iv2;
    const uint32_t e = (uint32_t)so + u;
    if (o.c) {
        st(o.c + m.c_soc, e, se - se0 - dt * (etac * sc - sd / etad));
        st(o.c + m.c_slp, e, ps + sd - sc - pls - rr * i2);
        st(o.c + m.c_slq, e, qs - qsc - qls - xx * i2);
        st(o.c + m.c_sth, e, S2 - rat * rat);
        if (m.comp) st(o.c + m.c_scmp, e, sc * sd);
    }
    if (o.J) {
        // columns ascending: soc [se_prev], se, sc, sd; loss_p vm, ps, qs, sc,
        // sd; loss_q vm, ps, qs, qsc; thermal ps, qs; comp sc, sd
        if (r >= 1) {
            const uint32_t j = (uint32_t)(3 * S + 4 * S * (r - 1)) + 4 * u;
            st(o.J + m.j_soc, j, -1.0);
            st(o.J + m.j_soc, j + 1, 1.0);
            st(o.J + m.j_soc, j + 2, -dt * etac);
            st(o.J + m.j_soc, j + 3, dt / etad);
        } else {
            st(o.J + m.j_soc, 3 * u, 1.0);
            st(o.J + m.j_soc, 3 * u + 1, -dt * etac);
            st(o.J + m.j_soc, 3 * u + 2, dt / etad);
        }
        const double dvm = 2.0 * S2 * iv3;  // d i2 / d vm = -dvm
        st(o.J + m.j_slp, 5 * e, rr * dvm);
        st(o.J + m.j_slp, 5 * e + 1, 1.0 - 2.0 * rr * ps * iv2);
        st(o.J + m.j_slp, 5 * e + 2, -2.0 * rr * qs * iv2);
        st(o.J + m.j_slp, 5 * e + 3, -1.0);
        st(o.J + m.j_slp, 5 * e + 4, 1.0);
        st(o.J + m.j_slq, 4 * e, xx * dvm);
        st(o.J + m.j_slq, 4 * e + 1, -2.0 * xx * ps * iv2);
        st(o.J + m.j_slq, 4 * e + 2, 1.0 - 2.0 * xx * qs * iv2);
        st(o.J + m.j_slq, 4 * e + 3, -1.0);
        st(o.J + m.j_sth, 2 * e, 2.0 * ps);
        st(o.J + m.j_sth, 2 * e + 1, 2.0 * qs);
        if (m.comp) {
            st(o.J + m.j_scmp, 2 * e, sd);
            st(o.J + m.j_scmp, 2 * e + 1, sc);
        }
    }
    if (o.H) {
        // the loss rows weigh -i2 by w; d2 i2 / dps2 = 2 / vm^2,
        // d2 i2 / (dps dvm) = -4 ps / vm^3
        const double w = ylp * rr + ylq * xx;
        st(o.H + m.h_ps, 2 * e, 4.0 * w * ps * iv3);
        st(o.H + m.h_ps, 2 * e + 1, -2.0 * w * iv2 + 2.0 * yth);
        st(o.H + m.h_qs, 2 * e, 4.0 * w * qs * iv3);
        st(o.H + m.h_qs, 2 * e + 1, -2.0 * w * iv2 + 2.0 * yth);
        if (m.comp) st(o.H + m.h_sd, e, ycm);
    }
    if (o.g) {
        st(o.g + m.x_ps + so, u, 0.0);
        st(o.g + m.x_qs + so, u, 0.0);
        st(o.g + m.x_qsc + so, u, 0.0);
        st(o.g + m.x_se + so, u, 0.0);
        st(o.g + m.x_sc + so, u, 0.0);
        st(o.g + m.x_sd + so, u, 0.0);
    }
}

// User-extension devices (Sec. III-D), one lane per device and replica:
// the gradient (cost), the ramp row (t >= 1) or the initial row (t = 0) and
// the device chunk's objective partial.  Balance entries: the bus segment.
template <bool SINGLE>
__device__ void dev_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const uint32_t d = (uint32_t)(chunk * kBlock) + threadIdx.x;
    const bool act = d < (uint32_t)m.D;
    const int64_t D = m.D, od = D * r;
    double fk = 0.0;
    if (act) {
        const double u = ld(o.x + m.x_u + od, d);
        const double cost = ld(m.dev_par + DP_COST * D, d);
        const double up = r >= 1 ? ld(o.x + m.x_u + od - D, d) : 0.0;
        fk = cost * u;
        if (o.g) st(o.g + m.x_u + od, d, cost);
        if (r >= 1) {
            const uint32_t e = (uint32_t)(D * (r - 1)) + d;
            if (o.c) st(o.c + m.c_dramp, e, u - up);
            if (o.J) {
                st(o.J + m.j_dramp, 2 * e, -1.0);
                st(o.J + m.j_dramp, 2 * e + 1, 1.0);
            }
        } else {
            if (o.c) st(o.c + m.c_dinit, d, u);
            if (o.J) st(o.J + m.j_dinit, d, 1.0);
        }
    }
    if (o.f) obj_partial<SINGLE, true>(m, o, (int64_t)m.ngchunks * m.npg + chunk + (int64_t)m.ndchunks * r, fk);
}

// J^T v of the storage units: each unit's six variable entries (its rows
// and its balance-row entries +1 on ps, qs).
__device__ void jt_stor_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const uint32_t u = (uint32_t)(chunk * kBlock) + threadIdx.x;
    if (u >= (uint32_t)m.S) return;
    const int64_t S = m.S, so = S * r, on = (int64_t)m.N * r;
    const double* P = m.stor_par;
    const double* x = o.x;
    const double* v = o.y;
    const uint32_t bus = (uint32_t)ld(m.stor_bus, u);
    const double ps = ld(x + m.x_ps + so, u), qs = ld(x + m.x_qs + so, u);
    const double sc = ld(x + m.x_sc + so, u), sd = ld(x + m.x_sd + so, u);
    const double vm = ld(x + m.x_vm + on, bus);
    const double etac = ld(P + SP_ETAC * S, u), etad = ld(P + SP_ETAD * S, u);
    const double rr = ld(P + SP_R * S, u), xx = ld(P + SP_X * S, u);
    const double vsoc = ld(v + m.c_soc + so, u);
    const double vsoc1 = (r + 1 < m.nrep) ? ld(v + m.c_soc + so + S, u) : 0.0;
    const double vlp = ld(v + m.c_slp + so, u), vlq = ld(v + m.c_slq + so, u), vth = ld(v + m.c_sth + so, u);
    const double vcm = m.comp ? ld(v + m.c_scmp + so, u) : 0.0;
    const double vbp = ld(v + m.c_balp + on, bus), vbq = ld(v + m.c_balq + on, bus);
    const double iv2 = 1.0 / (vm * vm), dt = m.stor_dt;
    st(o.g + m.x_ps + so, u, vlp * (1.0 - 2.0 * rr * ps * iv2) - vlq * 2.0 * xx * ps * iv2 + 2.0 * ps * vth + vbp);
    st(o.g + m.x_qs + so, u, -vlp * 2.0 * rr * qs * iv2 + vlq * (1.0 - 2.0 * xx * qs * iv2) + 2.0 * qs * vth + vbq);
    st(o.g + m.x_qsc + so, u, -vlq);
    st(o.g + m.x_se + so, u, vsoc - vsoc1);
    st(o.g + m.x_sc + so, u, -dt * etac * vsoc - vlp + vcm * sd);
    st(o.g + m.x_sd + so, u, dt / etad * vsoc + vlp + vcm * sc);
}

// J^T v of the devices: balance coefficients, ramp and initial rows.
__device__ void jt_dev_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const uint32_t d = (uint32_t)(chunk * kBlock) + threadIdx.x;
    if (d >= (uint32_t)m.D) return;
    const int64_t D = m.D, od = D * r, on = (int64_t)m.N * r;
    const double* v = o.y;
    const uint32_t bus = (uint32_t)ld(m.dev_bus, d);
    const double cp = ld(m.dev_par + DP_CP * D, d), cq = ld(m.dev_par + DP_CQ * D, d);
    const double vbp = ld(v + m.c_balp + on, bus), vbq = ld(v + m.c_balq + on, bus);
    // u_r enters the ramp row of period r (+1), of period r + 1 (-1) and,
    // at r = 0, the initial row
    const double own = r >= 1 ? ld(v + m.c_dramp + od - D, d) : ld(v + m.c_dinit, d);
    const double next = (r + 1 < m.nrep) ? ld(v + m.c_dramp + od, d) : 0.0;
    st(o.g + m.x_u + od, d, cp * vbp + cq * vbq + own - next);
}

}  // namespace

// ================================================================== dispatch
// Every work item covers one replica: a loop over replicas inside an item
// lets the compiler turn each output stream into its own per-lane 64-bit
// pointer (more than doubling the branch task's registers).
// RECT selects the rectangular form's tasks (every kernel is instantiated
// for both forms; a launch takes the model's).
template <int MODE, bool RECT, bool EXT>
__device__ __forceinline__ void run_phase1(const DevModel& m, const EvalOut& o, int32_t kind, int32_t idx, int32_t r,
                                           double* stage) {
    if (MODE == 0) {
        if (kind == T_GEN)
            gen_task<false, RECT, EXT>(m, o, idx, r);
        else if (EXT && kind == T_STOR)
            stor_task(m, o, idx, r);
        else if (EXT && kind == T_DEV)
            dev_task<false>(m, o, idx, r);
        else if (RECT)
            rbranch_task<false>(m, o, idx, r, stage);
        else
            branch_task<false>(m, o, idx, r, stage);
    } else if (MODE == 1) {
        if (EXT && kind == T_STOR)
            jt_stor_task(m, o, idx, r);
        else if (EXT && kind == T_DEV)
            jt_dev_task(m, o, idx, r);
        else if (RECT)
            rjt_branch_task(m, o, idx, r);
        else
            jt_branch_task(m, o, idx, r);
    } else if (kind == T_BRANCH) {
        flows_task(m, o, idx, r);
    }
}

template <int MODE, bool RECT, bool EXT>
__device__ __forceinline__ void run_phase2(const DevModel& m, const EvalOut& o, int32_t kind, int32_t idx, int32_t r,
                                           double* lds) {
    if (MODE == 0) {
        switch (kind) {
        case T_BIG: big_task<false, RECT, EXT>(m, o, idx, r); break;
        case T_WAVE: wave_task<false, RECT, EXT>(m, o, idx, r, lds); break;
        default: obj_task<EXT>(m, o); break;
        }
    } else {
        switch (kind) {
        case T_BIG: jt_big_task<RECT, EXT>(m, o, idx, r); break;
        case T_WAVE: jt_wave_task<RECT, EXT>(m, o, idx, r, lds); break;
        default: jt_gen_task(m, o, idx, r); break;
        }
    }
}

// Item b of a plain launch; replicas outermost, so one XCD's contiguous
// item range covers neighbouring entities of the same replicas.
template <bool EXT>
__device__ __forceinline__ void decode_phase1(const SetGrid& g, const DevModel& m, int32_t b, int32_t& kind,
                                              int32_t& idx, int32_t& r) {
    if (b < g.n_branch) {
        kind = T_BRANCH;
        idx = b % m.nbchunks;
        r = b / m.nbchunks;
    } else if ((b -= g.n_branch) < g.n_gen1 || !EXT) {
        kind = T_GEN;
        idx = b % m.ngchunks;
        r = b / m.ngchunks;
    } else if ((b -= g.n_gen1) < g.n_stor) {
        kind = T_STOR;
        idx = b % m.nschunks;
        r = b / m.nschunks;
    } else {
        b -= g.n_stor;
        kind = T_DEV;
        idx = b % m.ndchunks;
        r = b / m.ndchunks;
    }
}

__device__ __forceinline__ void decode_phase2(const SetGrid& g, const DevModel& m, int32_t b, int32_t& kind,
                                              int32_t& idx, int32_t& r) {
    int32_t per;
    if (b < g.n_big) {
        kind = T_BIG;
        per = m.nbig;
    } else if ((b -= g.n_big) < g.n_wave) {
        kind = T_WAVE;
        per = m.nwaves;
    } else if ((b -= g.n_wave) < g.n_obj) {
        kind = T_OBJ;
        idx = r = 0;
        return;
    } else {
        b -= g.n_obj;
        kind = T_GEN;
        if (g.gen_per_item) {  // one generator per wave, all replicas
            idx = b;
            r = 0;
            return;
        }
        per = m.ngchunks;
    }
    idx = b % per;
    r = b / per;
}

template <int MODE, bool RECT, bool EXT>
__global__ void __launch_bounds__(kBlock, 6) branch_kernel(DevModel m, EvalOut o, SetGrid g) {
    __shared__ double stage[kRecStride * kBlock];
    int32_t kind, idx, r;
    decode_phase1<EXT>(g, m, xcd_item(blockIdx.x, gridDim.x), kind, idx, r);
    run_phase1<MODE, RECT, EXT>(m, o, kind, idx, r, stage);
}

// The single launch of a small model's callback set: items ordered branch
// chunks, generator chunks, big buses, waves (bus items recompute their
// half-edge terms, the generator items sum the objective by ticket, so no
// item waits for another).  Blocks are dealt to the XCDs round-robin, which
// spreads every kind of item over all of them: a small launch is bound by
// latency, not by the lines that neighbouring items share.
template <bool RECT, bool EXT>
__global__ void __launch_bounds__(kBlock) set_kernel_single(DevModel m, EvalOut o, SetGrid g) {
    __shared__ double lds[kRecStride * kBlock];
    int32_t b = blockIdx.x;
    if (b < g.n_branch) {
        if (RECT)
            rbranch_task<true>(m, o, b % m.nbchunks, b / m.nbchunks, lds);
        else
            branch_task<true>(m, o, b % m.nbchunks, b / m.nbchunks, lds);
        return;
    }
    b -= g.n_branch;
    if (b < g.n_gen1) {
        gen_task<true, RECT, EXT>(m, o, b % m.ngchunks, b / m.ngchunks);
        return;
    }
    b -= g.n_gen1;
    if constexpr (EXT) {
        if (b < g.n_stor) {
            stor_task(m, o, b % m.nschunks, b / m.nschunks);
            return;
        }
        b -= g.n_stor;
        if (b < g.n_dev) {
            dev_task<true>(m, o, b % m.ndchunks, b / m.ndchunks);
            return;
        }
        b -= g.n_dev;
    }
    if (b < g.n_big) {
        big_task<true, RECT, EXT>(m, o, b % m.nbig, b / m.nbig);
        return;
    }
    b -= g.n_big;
    wave_task<true, RECT, EXT>(m, o, b % m.nwaves, b / m.nwaves, lds);
}

template <int MODE, bool RECT, bool EXT>
__global__ void __launch_bounds__(kBlock, 6) bus_kernel(DevModel m, EvalOut o, SetGrid g) {
    __shared__ double lds[kRecStride * kBlock];
    int32_t kind, idx, r;
    decode_phase2(g, m, xcd_item(blockIdx.x, gridDim.x), kind, idx, r);
    run_phase2<MODE, RECT, EXT>(m, o, kind, idx, r, lds);
}

// Occupancy hints (second launch-bounds argument: waves per SIMD) are the
// highest that compile without register spills; the single-launch kernel
// keeps its registers (a small launch has few waves to hide latency with).
//
// Batch kernels, one per phase and mode, in two forms.  Persistent (a grid
// smaller than the item list): the list is split into kXcd contiguous
// ranges, one per XCD, and the workgroups of an XCD stride through their
// range, so no queue counter is needed and neighbouring items share an L2.
// Flat (one workgroup per item, no loop, so fewer registers): the block
// index is remapped to the same XCD ranges.
// The kernel's MODE equals a.mode for every launch that runs items (the bus
// phase of the flows mode has none).  Taking the mode from the template
// leaves one assignment per field: a branch on a.mode made the compiler
// keep this struct in private (scratch) memory.
template <int MODE>
__device__ __forceinline__ EvalOut batch_out(const BatchArgs& a, const BatchInst& bi, int32_t inst) {
    EvalOut o;
    o.single = 0;  // batches always take the two-launch shape (records, objective items)
    o.x = a.X + bi.xoff;
    if constexpr (MODE == 0) {
        o.y = a.Y ? a.Y + bi.coff : nullptr;
        o.sigma = a.sigma ? a.sigma[inst] : 0.0;
        o.f = a.F ? a.F + inst : nullptr;
        o.g = a.G ? a.G + bi.xoff : nullptr;
        o.c = a.C ? a.C + bi.coff : nullptr;
        o.J = a.J ? a.J + bi.joff : nullptr;
        o.H = a.H ? a.H + bi.hoff : nullptr;
    } else {  // J^T v (Y holds V, G holds OUT) or flows (G is X, written in place)
        o.y = MODE == 1 ? a.Y + bi.coff : nullptr;
        o.sigma = 0.0;
        o.f = nullptr;
        o.c = nullptr;
        o.J = nullptr;
        o.H = nullptr;
        o.g = a.G + bi.xoff;
    }
    return o;
}

__device__ __forceinline__ void xcd_stride(int32_t n, int32_t& first, int32_t& step, int32_t& end) {
    const int32_t P = gridDim.x, b = blockIdx.x;
    const int32_t x = b % kXcd;
    step = (P - x + kXcd - 1) / kXcd;  // workgroups on this XCD
    first = (int32_t)((int64_t)n * x / kXcd) + b / kXcd;
    end = (int32_t)((int64_t)n * (x + 1) / kXcd);
}

template <int MODE, bool RECT, bool EXT>
__global__ void __launch_bounds__(kBlock) batch_branch_kernel(BatchArgs a) {
    __shared__ double stage[kRecStride * kBlock];
    int32_t it, step, end;
    xcd_stride(a.n_items, it, step, end);
    for (; it < end; it += step) {
        const BatchItem w = a.items[it];
        const BatchInst& bi = a.inst[w.inst];
        run_phase1<MODE, RECT, EXT>(bi.m, batch_out<MODE>(a, bi, w.inst), w.kind, w.idx, w.r, stage);
    }
}

template <int MODE, bool RECT, bool EXT>
__global__ void __launch_bounds__(kBlock) batch_bus_kernel(BatchArgs a) {
    __shared__ double lds[kRecStride * kBlock];
    int32_t it, step, end;
    xcd_stride(a.n_items, it, step, end);
    for (; it < end; it += step) {
        const BatchItem w = a.items[it];
        const BatchInst& bi = a.inst[w.inst];
        run_phase2<MODE, RECT, EXT>(bi.m, batch_out<MODE>(a, bi, w.inst), w.kind, w.idx, w.r, lds);
        __syncthreads();
    }
}

template <int MODE, bool RECT, bool EXT>
__global__ void __launch_bounds__(kBlock) batch_branch_flat(BatchArgs a) {
    __shared__ double stage[kRecStride * kBlock];
    const int32_t it = xcd_item(blockIdx.x, gridDim.x);
    if (it >= a.n_items) return;
    const BatchItem w = a.items[it];
    const BatchInst& bi = a.inst[w.inst];
    // a local copy: the instance's fields load together at the start instead
    // of one dependent scalar round trip per branch that first uses them
    // (64-scenario batch: 97.5 -> 95.4 us)
    const DevModel mloc = bi.m;
    run_phase1<MODE, RECT, EXT>(mloc, batch_out<MODE>(a, bi, w.inst), w.kind, w.idx, w.r, stage);
}

template <int MODE, bool RECT, bool EXT>
__global__ void __launch_bounds__(kBlock, 5) batch_bus_flat(BatchArgs a) {
    __shared__ double lds[kRecStride * kBlock];
    const int32_t it = xcd_item(blockIdx.x, gridDim.x);
    if (it >= a.n_items) return;
    const BatchItem w = a.items[it];
    const BatchInst& bi = a.inst[w.inst];
    // a local copy: the instance's fields load together at the start instead
    // of one dependent scalar round trip per branch that first uses them
    // (64-scenario batch: 97.5 -> 95.4 us)
    const DevModel mloc = bi.m;
    run_phase2<MODE, RECT, EXT>(mloc, batch_out<MODE>(a, bi, w.inst), w.kind, w.idx, w.r, lds);
}

// The one-launch shape over a batch: one workgroup per item (in list order,
// dealt round-robin to the XCDs like the plain one-launch kernel), every
// task in its one-launch form.
template <bool RECT, bool EXT>
__global__ void __launch_bounds__(kBlock) batch_single_flat(BatchArgs a) {
    __shared__ double lds[kRecStride * kBlock];
    const int32_t it = blockIdx.x;
    if (it >= a.n_items) return;
    const BatchItem w = a.items[it];
    const BatchInst& bi = a.inst[w.inst];
    const DevModel m = bi.m;
    EvalOut o = batch_out<0>(a, bi, w.inst);
    o.single = 1;
    switch (w.kind) {
    case T_BRANCH:
        if (RECT)
            rbranch_task<true>(m, o, w.idx, w.r, lds);
        else
            branch_task<true>(m, o, w.idx, w.r, lds);
        break;
    case T_GEN: gen_task<true, RECT, EXT>(m, o, w.idx, w.r); break;
    case T_STOR:
        if (EXT) stor_task(m, o, w.idx, w.r);
        break;
    case T_DEV:
        if (EXT) dev_task<true>(m, o, w.idx, w.r);
        break;
    case T_BIG: big_task<true, RECT, EXT>(m, o, w.idx, w.r); break;
    default: wave_task<true, RECT, EXT>(m, o, w.idx, w.r, lds); break;
    }
}

SetGrid plan_set(const DevModel& m, const EvalOut& o, int32_t mode) {
    SetGrid g{};
    const bool any = mode == 1 || o.g || o.c || o.J || o.H;
    g.n_branch = any ? m.nbchunks * m.nrep : 0;
    if (mode == 0 && (any || o.f)) g.n_gen1 = m.ngchunks * (any ? m.nrep : m.npg);  // f alone: pg replicas
    g.n_stor = any ? m.nschunks * m.nrep : 0;
    g.n_dev = (any || (mode == 0 && o.f)) ? m.ndchunks * m.nrep : 0;  // f alone: the devices' cost terms
    g.n_big = any ? m.nbig * m.nrep : 0;
    g.n_wave = any ? m.nwaves * m.nrep : 0;
    g.n_obj = (mode == 0 && o.f && !o.single) ? 1 : 0;  // a single launch sums f by ticket
    if (mode == 1) {
        g.gen_per_item = (m.npg == 1 && m.nrep > 1) ? 1 : 0;
        g.n_gen2 = g.gen_per_item ? m.G : m.ngchunks * m.nrep;
    }
    return g;
}

// The form (RECT) and the presence of storage units or devices (EXT) pick
// the kernel instantiation.
bool has_ext(const DevModel& m) { return m.S > 0 || m.D > 0; }

template <bool RECT, bool EXT>
hipError_t launch_set_form(const DevModel& m, const EvalOut& o, hipStream_t stream) {
    const SetGrid g = plan_set(m, o, 0);
    if (o.single) {
        const int32_t n = g.phase1() + g.phase2();
        if (n > 0) hipLaunchKernelGGL((set_kernel_single<RECT, EXT>), dim3(n), dim3(kBlock), 0, stream, m, o, g);
        return hipGetLastError();
    }
    if (g.phase1() > 0)
        hipLaunchKernelGGL((branch_kernel<0, RECT, EXT>), dim3(g.phase1()), dim3(kBlock), 0, stream, m, o, g);
    if (g.phase2() > 0)
        hipLaunchKernelGGL((bus_kernel<0, RECT, EXT>), dim3(g.phase2()), dim3(kBlock), 0, stream, m, o, g);
    return hipGetLastError();
}

hipError_t launch_eval_set(const DevModel& m, const EvalOut& o_in, hipStream_t stream) {
    EvalOut o = o_in;
    o.single = m.single;  // plain launches of small models take the single-launch shape
    if (has_ext(m))
        return m.rect ? launch_set_form<true, true>(m, o, stream) : launch_set_form<false, true>(m, o, stream);
    return m.rect ? launch_set_form<true, false>(m, o, stream) : launch_set_form<false, false>(m, o, stream);
}

template <bool RECT, bool EXT>
hipError_t launch_jt_form(const DevModel& m, const EvalOut& o, hipStream_t stream) {
    const SetGrid g = plan_set(m, o, 1);
    if (g.phase1() > 0)
        hipLaunchKernelGGL((branch_kernel<1, RECT, EXT>), dim3(g.phase1()), dim3(kBlock), 0, stream, m, o, g);
    if (g.phase2() > 0)
        hipLaunchKernelGGL((bus_kernel<1, RECT, EXT>), dim3(g.phase2()), dim3(kBlock), 0, stream, m, o, g);
    return hipGetLastError();
}

hipError_t launch_jtprod(const DevModel& m, const double* x, const double* v, double* out, hipStream_t stream) {
    EvalOut o{};
    o.x = x;
    o.y = v;
    o.g = out;
    if (has_ext(m))
        return m.rect ? launch_jt_form<true, true>(m, o, stream) : launch_jt_form<false, true>(m, o, stream);
    return m.rect ? launch_jt_form<true, false>(m, o, stream) : launch_jt_form<false, false>(m, o, stream);
}

template <bool RECT, bool EXT>
void* batch_kernel_form(int phase, int mode, bool flat) {
    if (flat) {
        if (phase == 0) {
            if (mode == 0) return reinterpret_cast<void*>(&batch_branch_flat<0, RECT, EXT>);
            if (mode == 1) return reinterpret_cast<void*>(&batch_branch_flat<1, RECT, EXT>);
            return reinterpret_cast<void*>(&batch_branch_flat<2, RECT, EXT>);
        }
        return mode == 0 ? reinterpret_cast<void*>(&batch_bus_flat<0, RECT, EXT>)
                         : reinterpret_cast<void*>(&batch_bus_flat<1, RECT, EXT>);
    }
    if (phase == 0) {
        if (mode == 0) return reinterpret_cast<void*>(&batch_branch_kernel<0, RECT, EXT>);
        if (mode == 1) return reinterpret_cast<void*>(&batch_branch_kernel<1, RECT, EXT>);
        return reinterpret_cast<void*>(&batch_branch_kernel<2, RECT, EXT>);
    }
    return mode == 0 ? reinterpret_cast<void*>(&batch_bus_kernel<0, RECT, EXT>)
                     : reinterpret_cast<void*>(&batch_bus_kernel<1, RECT, EXT>);
}

void* batch_single_fn(bool rect, bool ext) {
    if (ext)
        return rect ? reinterpret_cast<void*>(&batch_single_flat<true, true>)
                    : reinterpret_cast<void*>(&batch_single_flat<false, true>);
    return rect ? reinterpret_cast<void*>(&batch_single_flat<true, false>)
                : reinterpret_cast<void*>(&batch_single_flat<false, false>);
}

void* batch_kernel_fn(int phase, int mode, bool flat, bool rect, bool ext) {
    if (ext) return rect ? batch_kernel_form<true, true>(phase, mode, flat) : batch_kernel_form<false, true>(phase, mode, flat);
    return rect ? batch_kernel_form<true, false>(phase, mode, flat) : batch_kernel_form<false, false>(phase, mode, flat);
}

size_t scratch_bytes(const DevModel& m) {
    const size_t parts = ((sizeof(double) * (size_t)obj_slots(m)) + 255) & ~size_t(255);
    return parts + 256 + sizeof(double) * (size_t)kRecStride * 2 * m.nrep * m.L;
}

}  // namespace opf
