// gfx950 kernels for the polar AC-OPF callbacks (f, grad f, c, J, H) and
// the vector-Jacobian product J^T v.
//
// Every output entry is written exactly once by the work item that owns it,
// with no floating-point atomics; every sum runs in an order fixed by the
// model, so every launch shape (plain grid, persistent batch, any replica
// grouping) gives bitwise the same results.
//
// A callback set runs in two phases, each a 64-lane-workgroup launch, and
// each phase writes only outputs laid out in its own order, so every store
// of a wave lands in a few contiguous runs (no scattered partial-line
// writes, which the per-XCD L2s would each write back separately):
//  phase 1, branch items (one lane per branch, branch order, so branch data,
//    multipliers and arc variables are read coalesced; only the four bus
//    voltages are gathered): the four flow rows, the angle row and the two
//    thermal rows (c, J), the arc Hessian diagonals, and one 48-byte record
//    per half-edge (the weighted second derivatives of the branch's flow
//    rows and the arc's p, q), written contiguously in branch order;
//  phase 2, bus items: waves of packed bus segments [head, half-edges,
//    generators] (the host packs them so no segment straddles a wave and
//    precomputes every lane's output positions).  Each half-edge lane reads
//    its record (one aligned 48-byte gather), stages it in LDS, and the
//    head lane reduces its segment in order (a segmented reduction) into the
//    balance rows and the bus's Hessian diagonal, while the first half-edge
//    of each neighbour group writes the group's off-diagonal Hessian
//    entries (parallel branches summed); all of these sit in the bus's own
//    Hessian rows.  Buses wider than a wave are reduced by a whole
//    workgroup; generator items write the gradient, the pg Hessian
//    diagonal, reference and ramp rows, and one objective partial per
//    (chunk, replica) -- the chunk whose arrival completes a self-resetting
//    ticket sums the partials in index order.
// Workgroups are dealt to the 8 XCDs round-robin; both launches remap the
// block index so that each XCD takes a contiguous range of work items, and
// the cache lines that neighbouring items share meet in one L2.
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

namespace opf {

namespace {

// slot kinds (host_model.h)
constexpr int32_t SK_HEAD = 1, SK_EDGE = 2, SK_GEN = 3;

struct Coef {
    double Gff, Bff, Gft, Bft, Gtt, Btt, Gtf, Btf;
};

__device__ __forceinline__ Coef load_coef(const DevModel& m, int32_t l) {
    const size_t L = (size_t)m.L;
    const double* c = m.coef;
    return Coef{c[l], c[L + l], c[2 * L + l], c[3 * L + l], c[4 * L + l], c[5 * L + l], c[6 * L + l], c[7 * L + l]};
}

// A branch out of service in a contingency copy has zero admittance terms.
__device__ __forceinline__ Coef in_service(const Coef& k, const DevModel& m, int32_t l, int32_t r) {
    return m.outage[r] == l ? Coef{0, 0, 0, 0, 0, 0, 0, 0} : k;
}

// Half-edge record of (replica r, branch l, side s): kRec doubles, the two
// sides of a branch adjacent, branches in order.
__device__ __forceinline__ double* rec_at(const DevModel& m, int32_t r, int32_t l, int32_t side) {
    return m.rec + (((int64_t)r * m.L + l) * 2 + side) * kRec;
}
// The J^T v record: two doubles (va term, vm term) per half-edge.
__device__ __forceinline__ double* jt_rec_at(const DevModel& m, int32_t r, int32_t l, int32_t side) {
    return m.rec + (((int64_t)r * m.L + l) * 2 + side) * 2;
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
// weighted sum needs one trig evaluation.
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

__device__ __forceinline__ void put_flow_row(const EvalOut& o, int64_t row, int64_t jpos, double arcval,
                                             const Flow1& fl, bool f_lo) {
    if (o.c) o.c[row] = arcval - fl.F;
    if (o.J) {
        double* J = o.J + jpos;
        if (f_lo) {  // columns va_f, va_t, vm_f, vm_t, arc
            J[0] = -fl.Ft;
            J[1] = fl.Ft;
            J[2] = -fl.Fu;
            J[3] = -fl.Fw;
        } else {     // columns va_t, va_f, vm_t, vm_f, arc
            J[0] = fl.Ft;
            J[1] = -fl.Ft;
            J[2] = -fl.Fw;
            J[3] = -fl.Fu;
        }
        J[4] = 1.0;
    }
}

// ================================================================== phase 1
__device__ void branch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r0, int32_t r1) {
    const int32_t l = chunk * kBlock + (int32_t)threadIdx.x;
    if (l >= m.L) return;
    const int64_t L = m.L, N = m.N;
    const bool wantC = o.c != nullptr, wantJ = o.J != nullptr, wantH = o.H != nullptr;
    const bool wantFlow = wantC || wantJ || wantH;
    const int32_t fb = m.f_bus[l], tb = m.t_bus[l];
    const bool f_lo = fb < tb;
    Coef k0{};
    double rate2 = 0.0;
    if (wantFlow) {
        k0 = load_coef(m, l);
        if (wantC) rate2 = m.rate2[l];
    }
    const double* x = o.x;
    for (int32_t r = r0; r < r1; r++) {
        const int64_t rl = l + L * r;        // row inside a branch block
        const int64_t afr = l + 2 * L * r;   // from arc inside the p / q blocks
        const int64_t ato = afr + L;         // to arc
        if (wantFlow) {
            const double pf = x[m.x_p + afr], pt = x[m.x_p + ato];
            const double qf = x[m.x_q + afr], qt = x[m.x_q + ato];
            const Coef k = in_service(k0, m, l, r);
            const double u = x[m.x_vm + fb + N * r], w = x[m.x_vm + tb + N * r];
            const double vaf = x[m.x_va + fb + N * r], vat = x[m.x_va + tb + N * r];
            double S, C;
            sincos(vaf - vat, &S, &C);
            if (wantC || wantJ) {
                put_flow_row(o, m.c_pfr + rl, m.j_pfr + 5 * rl, pf, flow1(k.Gff, 0.0, k.Gft, k.Bft, u, w, C, S), f_lo);
                put_flow_row(o, m.c_qfr + rl, m.j_qfr + 5 * rl, qf, flow1(-k.Bff, 0.0, -k.Bft, k.Gft, u, w, C, S),
                             f_lo);
                put_flow_row(o, m.c_pto + rl, m.j_pto + 5 * rl, pt, flow1(0.0, k.Gtt, k.Gtf, -k.Btf, u, w, C, S), f_lo);
                put_flow_row(o, m.c_qto + rl, m.j_qto + 5 * rl, qt, flow1(0.0, -k.Btt, -k.Btf, -k.Gtf, u, w, C, S),
                             f_lo);
            }
            if (wantC) {
                o.c[m.c_ang + rl] = vaf - vat;
                o.c[m.c_thf + rl] = pf * pf + qf * qf - rate2;
                o.c[m.c_tht + rl] = pt * pt + qt * qt - rate2;
            }
            if (wantJ) {
                o.J[m.j_ang + 2 * rl] = f_lo ? 1.0 : -1.0;
                o.J[m.j_ang + 2 * rl + 1] = f_lo ? -1.0 : 1.0;
                o.J[m.j_thf + 2 * rl] = 2.0 * pf;
                o.J[m.j_thf + 2 * rl + 1] = 2.0 * qf;
                o.J[m.j_tht + 2 * rl] = 2.0 * pt;
                o.J[m.j_tht + 2 * rl + 1] = 2.0 * qt;
            }
            // the two half-edge records: [TT, MA, MM, UW, P, Q] at the from
            // side, then at the to side (12 doubles, 16-byte aligned)
            double2* rec = reinterpret_cast<double2*>(rec_at(m, r, l, 0));
            if (wantH) {
                const double yf = o.y[m.c_thf + rl], yt = o.y[m.c_tht + rl];
                o.H[m.h_p + afr] = 2.0 * yf;
                o.H[m.h_p + ato] = 2.0 * yt;
                o.H[m.h_q + afr] = 2.0 * yf;
                o.H[m.h_q + ato] = 2.0 * yt;
                const Hterms h = hess_terms(k, o.y[m.c_pfr + rl], o.y[m.c_qfr + rl], o.y[m.c_pto + rl],
                                            o.y[m.c_qto + rl], u, w, C, S);
                // d/dva_f = d/dth, d/dva_t = -d/dth
                rec[0] = make_double2(h.Stt, h.Sut);
                rec[1] = make_double2(h.Suu, h.Suw);
                rec[3] = make_double2(h.Stt, -h.Swt);
                rec[4] = make_double2(h.Sww, h.Suw);
            }
            if (wantC) {
                rec[2] = make_double2(pf, qf);
                rec[5] = make_double2(pt, qt);
            }
        }
        if (o.g) {
            o.g[m.x_p + afr] = 0.0;
            o.g[m.x_p + ato] = 0.0;
            o.g[m.x_q + afr] = 0.0;
            o.g[m.x_q + ato] = 0.0;
        }
    }
}

// J^T v, phase 1: the arc entries p / q (owned here) and each half-edge's
// va / vm terms for the bus side.
__device__ void jt_branch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r0, int32_t r1) {
    const int32_t l = chunk * kBlock + (int32_t)threadIdx.x;
    if (l >= m.L) return;
    const int64_t L = m.L, N = m.N;
    const int32_t fb = m.f_bus[l], tb = m.t_bus[l];
    const Coef k0 = load_coef(m, l);
    const double* x = o.x;
    const double* v = o.y;
    for (int32_t r = r0; r < r1; r++) {
        const int64_t rl = l + L * r;
        const int64_t afr = l + 2 * L * r, ato = afr + L;
        const int64_t bf = fb + N * r, bt = tb + N * r;
        const double vtf = v[m.c_thf + rl], vtt = v[m.c_tht + rl];
        const double v1 = v[m.c_pfr + rl], v2 = v[m.c_qfr + rl], v3 = v[m.c_pto + rl], v4 = v[m.c_qto + rl];
        // p_a sits in its flow row (+1), its bus's balance row (+1) and its
        // thermal row (2 p_a); q_a likewise
        o.g[m.x_p + afr] = v1 + v[m.c_balp + bf] + 2.0 * x[m.x_p + afr] * vtf;
        o.g[m.x_p + ato] = v3 + v[m.c_balp + bt] + 2.0 * x[m.x_p + ato] * vtt;
        o.g[m.x_q + afr] = v2 + v[m.c_balq + bf] + 2.0 * x[m.x_q + afr] * vtf;
        o.g[m.x_q + ato] = v4 + v[m.c_balq + bt] + 2.0 * x[m.x_q + ato] * vtt;
        const double u = x[m.x_vm + bf], w = x[m.x_vm + bt];
        const double th = x[m.x_va + bf] - x[m.x_va + bt];
        const Coef k = in_service(k0, m, l, r);
        double S, C;
        sincos(th, &S, &C);
        const Jterms j = jt_terms(k, v1, v2, v3, v4, u, w, C, S);
        const double va = v[m.c_ang + rl];
        // d th / d va_f = 1, d th / d va_t = -1; the angle row is va_f - va_t
        double2* rec = reinterpret_cast<double2*>(jt_rec_at(m, r, l, 0));
        rec[0] = make_double2(j.Dt + va, j.Du);
        rec[1] = make_double2(-j.Dt - va, j.Dw);
    }
}

// Arc variables := branch flows F(vm, va) (the x rows are read from o.x,
// the p / q entries written through o.g, which may alias it).
__device__ void flows_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r0, int32_t r1) {
    const int32_t l = chunk * kBlock + (int32_t)threadIdx.x;
    if (l >= m.L) return;
    const int64_t L = m.L, N = m.N;
    const int32_t fb = m.f_bus[l], tb = m.t_bus[l];
    const Coef k0 = load_coef(m, l);
    for (int32_t r = r0; r < r1; r++) {
        const int64_t afr = l + 2 * L * r, ato = afr + L;
        const Coef k = in_service(k0, m, l, r);
        const double u = o.x[m.x_vm + fb + N * r], w = o.x[m.x_vm + tb + N * r];
        const double th = o.x[m.x_va + fb + N * r] - o.x[m.x_va + tb + N * r];
        double S, C;
        sincos(th, &S, &C);
        o.g[m.x_p + afr] = flow1(k.Gff, 0.0, k.Gft, k.Bft, u, w, C, S).F;
        o.g[m.x_q + afr] = flow1(-k.Bff, 0.0, -k.Bft, k.Gft, u, w, C, S).F;
        o.g[m.x_p + ato] = flow1(0.0, k.Gtt, k.Gtf, -k.Btf, u, w, C, S).F;
        o.g[m.x_q + ato] = flow1(0.0, -k.Btt, -k.Btf, -k.Gtf, u, w, C, S).F;
    }
}

// ================================================================== phase 2
struct Slot {
    int32_t kind, ref, bus, other, jpos, h0, h1, h2;
};
__device__ __forceinline__ Slot load_slot(const DevModel& m, int32_t w) {
    const int4* p = reinterpret_cast<const int4*>(m.slots) + ((size_t)w * kBlock + threadIdx.x) * 2;
    const int4 a = p[0], b = p[1];
    return Slot{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}

__device__ void wave_task(const DevModel& m, const EvalOut& o, int32_t w, int32_t r0, int32_t r1, double* lds) {
    const int32_t lane = threadIdx.x;
    const Slot sl = load_slot(m, w);
    const int32_t type = sl.kind & 3;
    const int32_t side = (sl.kind & 4) ? 0 : 1;  // the half-edge sits at its branch's from bus
    const bool leader = sl.kind & 8;
    const int32_t len = (sl.kind >> 8) & 0xff;  // segment (head) or group (leader) length
    const bool wantC = o.c != nullptr, wantH = o.H != nullptr;
    const int64_t N = m.N, G = m.G;
    const double* x = o.x;
    double gs = 0.0, bs = 0.0;
    if (type == SK_HEAD) {
        gs = m.gs[sl.bus];
        bs = m.bs[sl.bus];
    }
    for (int32_t r = r0; r < r1; r++) {
        double v[kRec] = {0, 0, 0, 0, 0, 0};
        double vm_i = 0.0, base_p = 0.0, base_q = 0.0, shunt = 0.0;
        if (type == SK_HEAD) {
            vm_i = x[m.x_vm + sl.bus + N * r];
            if (wantC) {
                const int64_t ld = sl.bus + (int64_t)m.load_stride * r;
                base_p = m.pd[ld] + gs * vm_i * vm_i;
                base_q = m.qd[ld] - bs * vm_i * vm_i;
            }
            if (wantH) shunt = 2.0 * gs * o.y[m.c_balp + sl.bus + N * r] - 2.0 * bs * o.y[m.c_balq + sl.bus + N * r];
        } else if (type == SK_EDGE) {
            const double2* rec = reinterpret_cast<const double2*>(rec_at(m, r, sl.ref, side));
            if (wantH) {
                const double2 a = rec[0], b = rec[1];
                v[R_TT] = a.x;
                v[R_MA] = a.y;
                v[R_MM] = b.x;
                v[R_UW] = b.y;
            }
            if (wantC) {
                const double2 c = rec[2];
                v[R_P] = c.x;
                v[R_Q] = c.y;
            }
        } else if (type == SK_GEN) {
            if (wantC) {
                v[R_P] = -x[m.x_pg + sl.ref + G * (m.npg > 1 ? r : 0)];
                v[R_Q] = -x[m.x_qg + sl.ref + G * r];
            }
        }
        if (wantC || wantH) {
            for (int q = 0; q < kRec; q++) lds[q * kBlock + lane] = v[q];
            __syncthreads();
            if (type == SK_HEAD) {
                double sp = base_p, sq = base_q, daa = 0.0, dma = 0.0, dmm = 0.0;
                for (int32_t j = 1; j < len; j++) {  // the segment, in order
                    sp += lds[R_P * kBlock + lane + j];
                    sq += lds[R_Q * kBlock + lane + j];
                    daa += lds[R_TT * kBlock + lane + j];
                    dma += lds[R_MA * kBlock + lane + j];
                    dmm += lds[R_MM * kBlock + lane + j];
                }
                if (wantC) {
                    o.c[m.c_balp + sl.bus + N * r] = sp;
                    o.c[m.c_balq + sl.bus + N * r] = sq;
                }
                if (wantH) {
                    const int64_t hva = m.h_va + m.hva_rep * r, hvm = m.h_vm + m.hvm_rep * r;
                    if (sl.h0 >= 0) o.H[hva + sl.h0] = daa;
                    if (sl.h1 >= 0) o.H[hvm + sl.h1] = dma;
                    o.H[hvm + sl.h2] = dmm + shunt;
                }
            } else if (type == SK_EDGE && wantH && leader) {
                // the neighbour group (parallel branches to one bus), in order
                double tt = v[R_TT], ma = v[R_MA], uw = v[R_UW];
                for (int32_t j = 1; j < len; j++) {
                    tt += lds[R_TT * kBlock + lane + j];
                    ma += lds[R_MA * kBlock + lane + j];
                    uw += lds[R_UW * kBlock + lane + j];
                }
                const int64_t hva = m.h_va + m.hva_rep * r, hvm = m.h_vm + m.hvm_rep * r;
                if (sl.h0 >= 0) o.H[hva + sl.h0] = -tt;
                o.H[hvm + sl.h1] = -ma;
                if (sl.h2 >= 0) o.H[hvm + sl.h2] = uw;
            }
            __syncthreads();  // LDS is reused by the next replica
        }
        if (o.J) {
            const int64_t jp = m.j_balp + m.jbal_rep * r + sl.jpos, jq = m.j_balq + m.jbal_rep * r + sl.jpos;
            if (type == SK_HEAD) {
                o.J[jp] = 2.0 * gs * vm_i;
                o.J[jq] = -2.0 * bs * vm_i;
            } else if (type == SK_EDGE) {
                o.J[jp] = 1.0;
                o.J[jq] = 1.0;
            } else if (type == SK_GEN) {
                o.J[jp] = -1.0;
                o.J[jq] = -1.0;
            }
        }
        if (o.g && type == SK_HEAD) {
            o.g[m.x_va + sl.bus + N * r] = 0.0;
            o.g[m.x_vm + sl.bus + N * r] = 0.0;
        }
    }
}

// J^T v, phase 2: va / vm entries of the packed buses.
__device__ void jt_wave_task(const DevModel& m, const EvalOut& o, int32_t w, int32_t r0, int32_t r1, double* lds) {
    const int32_t lane = threadIdx.x;
    const Slot sl = load_slot(m, w);
    const int32_t type = sl.kind & 3;
    const int32_t side = (sl.kind & 4) ? 0 : 1;
    const int32_t len = (sl.kind >> 8) & 0xff;
    const int64_t N = m.N;
    const double* x = o.x;
    const double* v = o.y;
    for (int32_t r = r0; r < r1; r++) {
        double ga = 0.0, gm = 0.0;
        if (type == SK_EDGE) {
            const double2 t = *reinterpret_cast<const double2*>(jt_rec_at(m, r, sl.ref, side));
            ga = t.x;
            gm = t.y;
        }
        lds[0 * kBlock + lane] = ga;
        lds[1 * kBlock + lane] = gm;
        __syncthreads();
        if (type == SK_HEAD) {
            const int64_t bi = sl.bus + N * r;
            double sa = 0.0, sm = 0.0;
            for (int32_t j = 1; j < len; j++) {
                sa += lds[0 * kBlock + lane + j];
                sm += lds[1 * kBlock + lane + j];
            }
            for (int32_t q = m.ref_ptr[sl.bus]; q < m.ref_ptr[sl.bus + 1]; q++)
                sa += v[m.c_ref + m.ref_list[q] + (int64_t)m.R * r];
            const double vm = x[m.x_vm + bi];
            sm += 2.0 * m.gs[sl.bus] * vm * v[m.c_balp + bi] - 2.0 * m.bs[sl.bus] * vm * v[m.c_balq + bi];
            o.g[m.x_va + bi] = sa;
            o.g[m.x_vm + bi] = sm;
        }
        __syncthreads();
    }
}

// A bus whose segment does not fit a wave: the workgroup sums its
// half-edges' records (lane-strided, then a fixed wave tree).
__device__ void big_task(const DevModel& m, const EvalOut& o, int32_t idx, int32_t r0, int32_t r1) {
    const int32_t b = m.big_bus[idx];
    const int32_t e0 = m.adj_ptr[b], e1 = m.adj_ptr[b + 1], deg = e1 - e0;
    const int64_t N = m.N, G = m.G;
    const double* x = o.x;
    const bool wantH = o.H != nullptr, wantC = o.c != nullptr;
    const int32_t g0 = m.gen_ptr[b], ng = m.gen_ptr[b + 1] - g0;
    const double gs = m.gs[b], bs = m.bs[b];
    for (int32_t r = r0; r < r1; r++) {
        const int64_t bi = b + N * r;
        const double vm = x[m.x_vm + bi];
        if (wantC || wantH) {
            double sp = 0.0, sq = 0.0, daa = 0.0, dma = 0.0, dmm = 0.0;
            for (int32_t q = threadIdx.x; q < deg; q += kBlock) {
                const int32_t code = m.he[e0 + q];
                const double* rec = rec_at(m, r, code >> 1, (code & 1) ? 0 : 1);
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
                        const int32_t cq = m.he[q];
                        const double* rec = rec_at(m, r, cq >> 1, (cq & 1) ? 0 : 1);
                        tt += rec[R_TT];
                        ma += rec[R_MA];
                        uw += rec[R_UW];
                    }
                    if (k < b) {
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
                    const int64_t ld = b + (int64_t)m.load_stride * r;
                    double cp = m.pd[ld] + gs * vm * vm + sp, cq = m.qd[ld] - bs * vm * vm + sq;
                    const int64_t pgb = m.x_pg + G * (m.npg > 1 ? r : 0), qgb = m.x_qg + G * r;
                    for (int32_t q = 0; q < ng; q++) {
                        cp -= x[pgb + m.gen_list[g0 + q]];
                        cq -= x[qgb + m.gen_list[g0 + q]];
                    }
                    o.c[m.c_balp + bi] = cp;
                    o.c[m.c_balq + bi] = cq;
                }
                if (wantH) {
                    const double shunt = 2.0 * gs * o.y[m.c_balp + bi] - 2.0 * bs * o.y[m.c_balq + bi];
                    const int64_t hva = m.h_va + m.hva_rep * r + m.hva_off[b];
                    const int64_t hvm = m.h_vm + m.hvm_rep * r + m.hvm_off[b];
                    const int32_t nlo = m.nlo[b];
                    o.H[hva + nlo] = daa;
                    o.H[hvm + nlo] = dma;
                    o.H[hvm + m.ndist[b] + 1 + nlo] = dmm + shunt;
                }
            }
        }
        if (o.J) {
            double* Jp = o.J + m.j_balp + m.jbal_rep * r + m.jbal_off[b];
            double* Jq = o.J + m.j_balq + m.jbal_rep * r + m.jbal_off[b];
            for (int32_t q = threadIdx.x; q < 1 + ng + deg; q += kBlock) {
                Jp[q] = q == 0 ? 2.0 * gs * vm : (q <= ng ? -1.0 : 1.0);
                Jq[q] = q == 0 ? -2.0 * bs * vm : (q <= ng ? -1.0 : 1.0);
            }
        }
        if (o.g && threadIdx.x == 0) {
            o.g[m.x_va + bi] = 0.0;
            o.g[m.x_vm + bi] = 0.0;
        }
    }
}

__device__ void jt_big_task(const DevModel& m, const EvalOut& o, int32_t idx, int32_t r0, int32_t r1) {
    const int32_t b = m.big_bus[idx];
    const int32_t e0 = m.adj_ptr[b], deg = m.adj_ptr[b + 1] - e0;
    const int64_t N = m.N;
    const double* x = o.x;
    const double* v = o.y;
    for (int32_t r = r0; r < r1; r++) {
        double sa = 0.0, sm = 0.0;
        for (int32_t q = threadIdx.x; q < deg; q += kBlock) {
            const int32_t code = m.he[e0 + q];
            const double* rec = jt_rec_at(m, r, code >> 1, (code & 1) ? 0 : 1);
            sa += rec[0];
            sm += rec[1];
        }
        sa = wave_sum(sa);
        sm = wave_sum(sm);
        if (threadIdx.x == 0) {
            const int64_t bi = b + N * r;
            for (int32_t q = m.ref_ptr[b]; q < m.ref_ptr[b + 1]; q++) sa += v[m.c_ref + m.ref_list[q] + (int64_t)m.R * r];
            const double vm = x[m.x_vm + bi];
            sm += 2.0 * m.gs[b] * vm * v[m.c_balp + bi] - 2.0 * m.bs[b] * vm * v[m.c_balq + bi];
            o.g[m.x_va + bi] = sa;
            o.g[m.x_vm + bi] = sm;
        }
    }
}

// ------------------------------------------------------------------ generators
// Phase 1: per generator chunk the gradient, the pg Hessian diagonal, the
// reference and ramp rows, and one objective partial per replica (a fixed
// wave tree over the chunk), written with a plain store: the objective item
// of phase 2 reads the partials after the launch boundary.
__device__ void gen_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r0, int32_t r1) {
    const int32_t k = chunk * kBlock + (int32_t)threadIdx.x;
    const double* x = o.x;
    const int64_t G = m.G;
    double c2 = 0.0, c1 = 0.0, c0 = 0.0;
    if (k < m.G) {
        c2 = m.c2[k];
        c1 = m.c1[k];
        c0 = m.c0[k];
    }
    for (int32_t r = r0; r < r1; r++) {
        double fk = 0.0;
        if (k < m.G) {
            if (r < m.npg) {
                const int64_t col = m.x_pg + k + G * r;
                const double pg = x[col];
                fk = c2 * pg * pg + c1 * pg + c0;
                if (o.g) o.g[col] = 2.0 * c2 * pg + c1;
                if (o.H) o.H[m.h_pg + k + G * r] = 2.0 * o.sigma * c2;
            }
            if (o.g) o.g[m.x_qg + k + G * r] = 0.0;
            if (m.T > 1 && r >= 1) {
                const int64_t row = k + G * (r - 1);
                if (o.c) o.c[m.c_ramp + row] = x[m.x_pg + k + G * r] - x[m.x_pg + k + G * (r - 1)];
                if (o.J) {
                    o.J[m.j_ramp + 2 * row] = -1.0;
                    o.J[m.j_ramp + 2 * row + 1] = 1.0;
                }
            }
        }
        if (k < m.R) {
            const int64_t row = k + (int64_t)m.R * r;
            if (o.c) o.c[m.c_ref + row] = x[m.x_va + m.ref_bus[k] + (int64_t)m.N * r];
            if (o.J) o.J[m.j_ref + row] = 1.0;
        }
        if (o.f && r < m.npg) {
            const double s = wave_sum(fk);
            if (threadIdx.x == 0) m.obj_part[chunk + (int64_t)m.ngchunks * r] = s;
        }
    }
}

// Phase 2: f = the partials summed lane-strided in index order, then a
// fixed wave tree.
__device__ void obj_task(const DevModel& m, const EvalOut& o) {
    if (o.f == nullptr) return;
    const int32_t total = m.ngchunks * m.npg;
    double acc = 0.0;
    for (int32_t q = threadIdx.x; q < total; q += kBlock) acc += m.obj_part[q];
    acc = wave_sum(acc);
    if (threadIdx.x == 0) *o.f = acc;
}

__device__ void jt_gen_task(const DevModel& m, const EvalOut& o, int32_t idx, int32_t r0, int32_t r1) {
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
    const int32_t k = idx * kBlock + (int32_t)threadIdx.x;
    if (k >= m.G) return;
    const int32_t bus = m.gen_bus[k];
    for (int32_t r = r0; r < r1; r++) {
        o.g[m.x_qg + k + G * r] = -v[m.c_balq + bus + N * r];
        double acc = -v[m.c_balp + bus + N * r];
        if (m.T > 1) {
            if (r >= 1) acc += v[m.c_ramp + k + G * (r - 1)];
            if (r + 1 < m.T) acc -= v[m.c_ramp + k + G * r];
        }
        o.g[m.x_pg + k + G * r] = acc;
    }
}

}  // namespace

// ================================================================== dispatch
__device__ __forceinline__ void run_phase1(const DevModel& m, const EvalOut& o, int32_t mode, int32_t kind,
                                           int32_t idx, int32_t r0, int32_t r1) {
    if (kind == T_GEN) {
        if (mode == 0) gen_task(m, o, idx, r0, r1);
    } else if (mode == 0) {
        branch_task(m, o, idx, r0, r1);
    } else if (mode == 1) {
        jt_branch_task(m, o, idx, r0, r1);
    } else {
        flows_task(m, o, idx, r0, r1);
    }
}

__device__ __forceinline__ void run_phase2(const DevModel& m, const EvalOut& o, int32_t mode, int32_t kind,
                                           int32_t idx, int32_t r0, int32_t r1, double* lds) {
    if (mode == 0) {
        switch (kind) {
        case T_BIG: big_task(m, o, idx, r0, r1); break;
        case T_WAVE: wave_task(m, o, idx, r0, r1, lds); break;
        default: obj_task(m, o); break;
        }
    } else {
        switch (kind) {
        case T_BIG: jt_big_task(m, o, idx, r0, r1); break;
        case T_WAVE: jt_wave_task(m, o, idx, r0, r1, lds); break;
        default: jt_gen_task(m, o, idx, r0, r1); break;
        }
    }
}

__device__ __forceinline__ void decode_phase1(const SetGrid& g, const DevModel& m, int32_t b, int32_t& kind,
                                              int32_t& idx, int32_t& r0, int32_t& r1) {
    if (b < g.n_branch) {
        kind = T_BRANCH;
        idx = b % m.nbchunks;
        r0 = (b / m.nbchunks) * g.rg1;
        r1 = min(r0 + g.rg1, m.nrep);
    } else {
        b -= g.n_branch;
        kind = T_GEN;
        idx = b % m.ngchunks;
        r0 = (b / m.ngchunks) * g.rgg;
        r1 = min(r0 + g.rgg, g.gen_nrep);
    }
}

__device__ __forceinline__ void decode_phase2(const SetGrid& g, const DevModel& m, int32_t b, int32_t& kind,
                                              int32_t& idx, int32_t& r0, int32_t& r1) {
    int32_t per;
    if (b < g.n_big) {
        kind = T_BIG;
        per = m.nbig;
    } else if ((b -= g.n_big) < g.n_wave) {
        kind = T_WAVE;
        per = m.nwaves;
    } else if ((b -= g.n_wave) < g.n_obj) {
        kind = T_OBJ;
        idx = r0 = r1 = 0;
        return;
    } else {
        b -= g.n_obj;
        kind = T_GEN;
        if (g.gen_per_item) {  // one generator per wave, all replicas
            idx = b;
            r0 = 0;
            r1 = m.nrep;
            return;
        }
        per = m.ngchunks;
    }
    // replica groups outermost, so one XCD's contiguous item range covers
    // neighbouring entities of the same replicas
    idx = b % per;
    r0 = (b / per) * g.rg2;
    r1 = min(r0 + g.rg2, m.nrep);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) branch_kernel(DevModel m, EvalOut o, SetGrid g) {
    int32_t kind, idx, r0, r1;
    decode_phase1(g, m, xcd_item(blockIdx.x, gridDim.x), kind, idx, r0, r1);
    run_phase1(m, o, MODE, kind, idx, r0, r1);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) bus_kernel(DevModel m, EvalOut o, SetGrid g) {
    __shared__ double lds[kRec * kBlock];
    int32_t kind, idx, r0, r1;
    decode_phase2(g, m, xcd_item(blockIdx.x, gridDim.x), kind, idx, r0, r1);
    run_phase2(m, o, MODE, kind, idx, r0, r1, lds);
}

// Persistent batch kernels, one per phase: a fixed grid sized to the chip
// drains the item list.  Items are split into kXcd contiguous ranges, one per
// XCD, and the workgroups of an XCD stride through its range, so no queue
// counter is needed and neighbouring items share an L2.
__device__ __forceinline__ EvalOut batch_out(const BatchArgs& a, const BatchInst& bi, int32_t inst) {
    EvalOut o;
    o.x = a.X + bi.xoff;
    if (a.mode == 0) {
        o.y = a.Y ? a.Y + bi.coff : nullptr;
        o.sigma = a.sigma ? a.sigma[inst] : 0.0;
        o.f = a.F ? a.F + inst : nullptr;
        o.g = a.G ? a.G + bi.xoff : nullptr;
        o.c = a.C ? a.C + bi.coff : nullptr;
        o.J = a.J ? a.J + bi.joff : nullptr;
        o.H = a.H ? a.H + bi.hoff : nullptr;
    } else {  // J^T v (Y holds V, G holds OUT) or flows (G is X, written in place)
        o.y = a.mode == 1 ? a.Y + bi.coff : nullptr;
        o.sigma = 0.0;
        o.f = nullptr;
        o.c = o.J = o.H = nullptr;
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

__global__ void __launch_bounds__(kBlock) batch_branch_kernel(BatchArgs a) {
    int32_t it, step, end;
    xcd_stride(a.n_items, it, step, end);
    for (; it < end; it += step) {
        const BatchItem w = a.items[it];
        const BatchInst& bi = a.inst[w.inst];
        run_phase1(bi.m, batch_out(a, bi, w.inst), a.mode, w.kind, w.idx, w.r0, w.r1);
    }
}

__global__ void __launch_bounds__(kBlock) batch_bus_kernel(BatchArgs a) {
    __shared__ double lds[kRec * kBlock];
    int32_t it, step, end;
    xcd_stride(a.n_items, it, step, end);
    for (; it < end; it += step) {
        const BatchItem w = a.items[it];
        const BatchInst& bi = a.inst[w.inst];
        run_phase2(bi.m, batch_out(a, bi, w.inst), a.mode, w.kind, w.idx, w.r0, w.r1, lds);
        __syncthreads();
    }
}

namespace {
int32_t group_for(int32_t per_rep, int32_t nrep) {
    // enough replicas per item to keep the grid near 4096 workgroups
    const int64_t items = (int64_t)per_rep * nrep;
    int32_t rg = (int32_t)((items + 4095) / 4096);
    return rg < 1 ? 1 : (rg > nrep ? nrep : rg);
}
}  // namespace

SetGrid plan_set(const DevModel& m, const EvalOut& o, int32_t mode) {
    SetGrid g{};
    const bool any = mode == 1 || o.g || o.c || o.J || o.H;
    g.rg1 = group_for(m.nbchunks, m.nrep);
    g.n_branch = any ? m.nbchunks * ((m.nrep + g.rg1 - 1) / g.rg1) : 0;
    if (mode == 0 && (any || o.f)) {
        // the objective alone needs the pg replicas only
        g.gen_nrep = any ? m.nrep : m.npg;
        g.rgg = group_for(m.ngchunks, g.gen_nrep);
        g.n_gen1 = m.ngchunks * ((g.gen_nrep + g.rgg - 1) / g.rgg);
    }
    g.rg2 = group_for(m.nbig + m.nwaves, m.nrep);
    g.nrg2 = (m.nrep + g.rg2 - 1) / g.rg2;
    g.n_big = any ? m.nbig * g.nrg2 : 0;
    g.n_wave = any ? m.nwaves * g.nrg2 : 0;
    g.n_obj = (mode == 0 && o.f) ? 1 : 0;
    if (mode == 1) {
        g.gen_per_item = (m.npg == 1 && m.nrep > 1) ? 1 : 0;
        g.n_gen2 = g.gen_per_item ? m.G : m.ngchunks * g.nrg2;
    }
    return g;
}

hipError_t launch_eval_set(const DevModel& m, const EvalOut& o, hipStream_t stream) {
    const SetGrid g = plan_set(m, o, 0);
    if (g.phase1() > 0) hipLaunchKernelGGL(branch_kernel<0>, dim3(g.phase1()), dim3(kBlock), 0, stream, m, o, g);
    if (g.phase2() > 0) hipLaunchKernelGGL(bus_kernel<0>, dim3(g.phase2()), dim3(kBlock), 0, stream, m, o, g);
    return hipGetLastError();
}

hipError_t launch_jtprod(const DevModel& m, const double* x, const double* v, double* out, hipStream_t stream) {
    EvalOut o{};
    o.x = x;
    o.y = v;
    o.g = out;
    const SetGrid g = plan_set(m, o, 1);
    if (g.phase1() > 0) hipLaunchKernelGGL(branch_kernel<1>, dim3(g.phase1()), dim3(kBlock), 0, stream, m, o, g);
    if (g.phase2() > 0) hipLaunchKernelGGL(bus_kernel<1>, dim3(g.phase2()), dim3(kBlock), 0, stream, m, o, g);
    return hipGetLastError();
}

void* batch_kernel_fn(int phase) {
    return phase == 0 ? reinterpret_cast<void*>(&batch_branch_kernel) : reinterpret_cast<void*>(&batch_bus_kernel);
}

size_t scratch_bytes(const DevModel& m) {
    const size_t parts = ((sizeof(double) * (size_t)m.ngchunks * m.npg) + 255) & ~size_t(255);
    return parts + sizeof(double) * (size_t)kRec * 2 * m.nrep * m.L;
}

}  // namespace opf
