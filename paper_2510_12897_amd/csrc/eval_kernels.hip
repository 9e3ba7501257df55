// gfx950 kernels for the polar AC-OPF callbacks (f, grad f, c, J, H) and
// the vector-Jacobian product J^T v.
//
// Every output entry is written exactly once by the work item that owns it,
// with no floating-point atomics; every sum runs in an order fixed by the
// model, so every launch shape (plain grid, persistent batch, any replica
// grouping) gives bitwise the same results.
//
// A callback set runs in two phases, each a 64-lane-workgroup launch:
//  phase 1, branch items (one lane per branch, branch order, so branch data,
//    multipliers and arc variables are read coalesced; only the four bus
//    voltages are gathered): the four flow rows, the angle row and the two
//    thermal rows (c, J), the arc Hessian diagonals, the branch's
//    off-diagonal Hessian entries, and for each of its two half-edges the
//    bus-side terms (arc p and q, weighted second derivatives) written to a
//    scratch laid out in the bus-side order;
//  phase 2, bus items: waves of packed bus segments [head, half-edges,
//    generators] (the host packs them so no segment straddles a wave and
//    precomputes every lane's output positions).  Each lane reads its own
//    scratch entries (coalesced), stages them in LDS, and the head lane
//    reduces its segment in order (a segmented reduction) into the balance
//    rows and the bus's Hessian diagonal; buses wider than a wave are
//    reduced by a whole workgroup; generator items write the gradient, the
//    pg Hessian diagonal, reference and ramp rows, and one objective
//    partial per (chunk, replica) -- the chunk whose arrival completes a
//    self-resetting ticket sums the partials in index order.
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

__device__ __forceinline__ double* scr_at(const DevModel& m, int32_t row, int32_t r, int64_t s) {
    return m.scr + ((int64_t)row * m.nrep + r) * m.nscr + s;
}

__device__ __forceinline__ double coherent_load(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coherent_store(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    int32_t s_fr = 0, s_to = 0, hx0 = -1, hx1 = -1, hx2 = -1, hx3 = -1;
    if (wantC || wantH) {
        s_fr = m.br_scr[l];
        s_to = m.br_scr[L + l];
    }
    if (wantH) {
        hx0 = m.br_hx[l];
        hx1 = m.br_hx[L + l];
        hx2 = m.br_hx[2 * L + l];
        hx3 = m.br_hx[3 * L + l];
    }
    Coef k0{};
    double rate2 = 0.0;
    if (wantFlow) {
        k0 = load_coef(m, l);
        rate2 = m.rate2[l];
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
                // arc terms of the two balance rows
                *scr_at(m, S_P, r, s_fr) = pf;
                *scr_at(m, S_Q, r, s_fr) = qf;
                *scr_at(m, S_P, r, s_to) = pt;
                *scr_at(m, S_Q, r, s_to) = qt;
            }
            if (wantJ) {
                o.J[m.j_ang + 2 * rl] = f_lo ? 1.0 : -1.0;
                o.J[m.j_ang + 2 * rl + 1] = f_lo ? -1.0 : 1.0;
                o.J[m.j_thf + 2 * rl] = 2.0 * pf;
                o.J[m.j_thf + 2 * rl + 1] = 2.0 * qf;
                o.J[m.j_tht + 2 * rl] = 2.0 * pt;
                o.J[m.j_tht + 2 * rl + 1] = 2.0 * qt;
            }
            if (wantH) {
                const double yf = o.y[m.c_thf + rl], yt = o.y[m.c_tht + rl];
                o.H[m.h_p + afr] = 2.0 * yf;
                o.H[m.h_p + ato] = 2.0 * yt;
                o.H[m.h_q + afr] = 2.0 * yf;
                o.H[m.h_q + ato] = 2.0 * yt;
                const Hterms h = hess_terms(k, o.y[m.c_pfr + rl], o.y[m.c_qfr + rl], o.y[m.c_pto + rl],
                                            o.y[m.c_qto + rl], u, w, C, S);
                // bus-side diagonal terms: (va_i, va_i), (vm_i, va_i), (vm_i, vm_i)
                *scr_at(m, S_DAA, r, s_fr) = h.Stt;
                *scr_at(m, S_DMA, r, s_fr) = h.Sut;
                *scr_at(m, S_DMM, r, s_fr) = h.Suu;
                *scr_at(m, S_DAA, r, s_to) = h.Stt;
                *scr_at(m, S_DMA, r, s_to) = -h.Swt;
                *scr_at(m, S_DMM, r, s_to) = h.Sww;
                // off-diagonal: (va_f, va_t), (vm_f, vm_t), (vm_f, va_t), (vm_t, va_f)
                const int64_t hva = m.h_va + m.hva_rep * r, hvm = m.h_vm + m.hvm_rep * r;
                if (hx0 >= 0) {
                    o.H[hva + hx0] = -h.Stt;
                    o.H[hvm + hx1] = h.Suw;
                    o.H[hvm + hx2] = -h.Sut;
                    o.H[hvm + hx3] = h.Swt;
                } else {  // parallel branches: the bus side sums the group
                    *scr_at(m, S_XAA, r, s_fr) = -h.Stt;
                    *scr_at(m, S_XMA, r, s_fr) = -h.Sut;
                    *scr_at(m, S_XMM, r, s_fr) = h.Suw;
                    *scr_at(m, S_XAA, r, s_to) = -h.Stt;
                    *scr_at(m, S_XMA, r, s_to) = h.Swt;
                    *scr_at(m, S_XMM, r, s_to) = h.Suw;
                }
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
    const int32_t s_fr = m.br_scr[l], s_to = m.br_scr[L + l];
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
        *scr_at(m, S_P, r, s_fr) = j.Dt + va;
        *scr_at(m, S_Q, r, s_fr) = j.Du;
        *scr_at(m, S_P, r, s_to) = -j.Dt - va;
        *scr_at(m, S_Q, r, s_to) = j.Dw;
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
    const int64_t sidx = (int64_t)w * kBlock + lane;  // this lane's scratch entry
    const Slot sl = load_slot(m, w);
    const int32_t type = sl.kind & 3;
    const bool leader = sl.kind & 8;
    const bool grouped = sl.kind & 16;
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
        double v[S_ROWS] = {0, 0, 0, 0, 0, 0, 0, 0};
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
            if (wantC) {
                v[S_P] = *scr_at(m, S_P, r, sidx);
                v[S_Q] = *scr_at(m, S_Q, r, sidx);
            }
            if (wantH) {
                v[S_DAA] = *scr_at(m, S_DAA, r, sidx);
                v[S_DMA] = *scr_at(m, S_DMA, r, sidx);
                v[S_DMM] = *scr_at(m, S_DMM, r, sidx);
                if (grouped) {
                    v[S_XAA] = *scr_at(m, S_XAA, r, sidx);
                    v[S_XMA] = *scr_at(m, S_XMA, r, sidx);
                    v[S_XMM] = *scr_at(m, S_XMM, r, sidx);
                }
            }
        } else if (type == SK_GEN) {
            if (wantC) {
                v[S_P] = -x[m.x_pg + sl.ref + G * (m.npg > 1 ? r : 0)];
                v[S_Q] = -x[m.x_qg + sl.ref + G * r];
            }
        }
        if (wantC || wantH) {
            for (int q = 0; q < S_ROWS; q++) lds[q * kBlock + lane] = v[q];
            __syncthreads();
            if (type == SK_HEAD) {
                double sp = base_p, sq = base_q, daa = 0.0, dma = 0.0, dmm = 0.0;
                for (int32_t j = 1; j < len; j++) {  // the segment, in order
                    sp += lds[S_P * kBlock + lane + j];
                    sq += lds[S_Q * kBlock + lane + j];
                    daa += lds[S_DAA * kBlock + lane + j];
                    dma += lds[S_DMA * kBlock + lane + j];
                    dmm += lds[S_DMM * kBlock + lane + j];
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
            } else if (type == SK_EDGE && wantH && leader && grouped) {
                double xaa = v[S_XAA], xma = v[S_XMA], xmm = v[S_XMM];
                for (int32_t j = 1; j < len; j++) {  // parallel branches to one neighbour
                    xaa += lds[S_XAA * kBlock + lane + j];
                    xma += lds[S_XMA * kBlock + lane + j];
                    xmm += lds[S_XMM * kBlock + lane + j];
                }
                const int64_t hva = m.h_va + m.hva_rep * r, hvm = m.h_vm + m.hvm_rep * r;
                if (sl.h0 >= 0) o.H[hva + sl.h0] = xaa;
                o.H[hvm + sl.h1] = xma;
                if (sl.h2 >= 0) o.H[hvm + sl.h2] = xmm;
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
    const int64_t sidx = (int64_t)w * kBlock + lane;
    const Slot sl = load_slot(m, w);
    const int32_t type = sl.kind & 3;
    const int32_t len = (sl.kind >> 8) & 0xff;
    const int64_t N = m.N;
    const double* x = o.x;
    const double* v = o.y;
    for (int32_t r = r0; r < r1; r++) {
        double ga = 0.0, gm = 0.0;
        if (type == SK_EDGE) {
            ga = *scr_at(m, S_P, r, sidx);
            gm = *scr_at(m, S_Q, r, sidx);
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
// half-edges' scratch entries (lane-strided, then a fixed wave tree).
__device__ void big_task(const DevModel& m, const EvalOut& o, int32_t idx, int32_t r0, int32_t r1) {
    const int32_t b = m.big_bus[idx];
    const int32_t e0 = m.adj_ptr[b], e1 = m.adj_ptr[b + 1], deg = e1 - e0;
    const int32_t s0 = m.big_scr[idx];
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
                if (wantC) {
                    sp += *scr_at(m, S_P, r, s0 + q);
                    sq += *scr_at(m, S_Q, r, s0 + q);
                }
                if (wantH) {
                    daa += *scr_at(m, S_DAA, r, s0 + q);
                    dma += *scr_at(m, S_DMA, r, s0 + q);
                    dmm += *scr_at(m, S_DMM, r, s0 + q);
                }
            }
            sp = wave_sum(sp);
            sq = wave_sum(sq);
            daa = wave_sum(daa);
            dma = wave_sum(dma);
            dmm = wave_sum(dmm);
            if (wantH) {  // parallel-branch groups: the group's first half-edge sums it
                const int64_t hva = m.h_va + m.hva_rep * r + m.hva_off[b];
                const int64_t hvm = m.h_vm + m.hvm_rep * r + m.hvm_off[b];
                for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += kBlock) {
                    const int32_t grp = m.he_grp[e];
                    if (e > e0 && m.he_grp[e - 1] == grp) continue;
                    if (!(e + 1 < e1 && m.he_grp[e + 1] == grp)) continue;  // single branch: written in phase 1
                    const int32_t code = m.he[e], l = code >> 1;
                    const int32_t k = (code & 1) ? m.t_bus[l] : m.f_bus[l];
                    double xaa = 0.0, xma = 0.0, xmm = 0.0;
                    for (int32_t q = e; q < e1 && m.he_grp[q] == grp; q++) {
                        xaa += *scr_at(m, S_XAA, r, s0 + (q - e0));
                        xma += *scr_at(m, S_XMA, r, s0 + (q - e0));
                        xmm += *scr_at(m, S_XMM, r, s0 + (q - e0));
                    }
                    if (k < b) {
                        o.H[hva + grp] = xaa;
                        o.H[hvm + grp] = xma;
                        o.H[hvm + m.ndist[b] + 1 + grp] = xmm;
                    } else {
                        o.H[hvm + grp + 1] = xma;
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
    const int32_t deg = m.adj_ptr[b + 1] - m.adj_ptr[b];
    const int32_t s0 = m.big_scr[idx];
    const int64_t N = m.N;
    const double* x = o.x;
    const double* v = o.y;
    for (int32_t r = r0; r < r1; r++) {
        double sa = 0.0, sm = 0.0;
        for (int32_t q = threadIdx.x; q < deg; q += kBlock) {
            sa += *scr_at(m, S_P, r, s0 + q);
            sm += *scr_at(m, S_Q, r, s0 + q);
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
    int32_t parts = 0;
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
            if (threadIdx.x == 0) coherent_store(&m.obj_part[chunk + (int64_t)m.ngchunks * r], s);
            parts++;
        }
    }
    if (o.f && parts > 0) {
        // the chunk that brings the count to ngchunks * npg sums every partial
        __shared__ int32_t last;
        if (threadIdx.x == 0) {
            const int32_t total = m.ngchunks * m.npg;
            const int32_t old = __hip_atomic_fetch_add(m.obj_ticket, parts, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            last = (old + parts == total) ? 1 : 0;
        }
        __syncthreads();
        if (last) {
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
            const int32_t total = m.ngchunks * m.npg;
            double acc = 0.0;
            for (int32_t q = threadIdx.x; q < total; q += kBlock) acc += coherent_load(&m.obj_part[q]);
            acc = wave_sum(acc);
            if (threadIdx.x == 0) {
                *o.f = acc;
                __hip_atomic_store(m.obj_ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
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
__device__ void run_task(const DevModel& m, const EvalOut& o, int32_t mode, int32_t kind, int32_t idx, int32_t r0,
                         int32_t r1, double* lds) {
    if (mode == 2) {
        flows_task(m, o, idx, r0, r1);
    } else if (mode == 0) {
        switch (kind) {
        case T_BRANCH: branch_task(m, o, idx, r0, r1); break;
        case T_BIG: big_task(m, o, idx, r0, r1); break;
        case T_WAVE: wave_task(m, o, idx, r0, r1, lds); break;
        default: gen_task(m, o, idx, r0, r1); break;
        }
    } else {
        switch (kind) {
        case T_BRANCH: jt_branch_task(m, o, idx, r0, r1); break;
        case T_BIG: jt_big_task(m, o, idx, r0, r1); break;
        case T_WAVE: jt_wave_task(m, o, idx, r0, r1, lds); break;
        default: jt_gen_task(m, o, idx, r0, r1); break;
        }
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
    } else {
        b -= g.n_wave;
        kind = T_GEN;
        if (g.gen_per_item) {  // one generator per wave, all replicas
            idx = b;
            r0 = 0;
            r1 = m.nrep;
            return;
        }
        per = m.ngchunks;
    }
    idx = b % per;
    r0 = (b / per) * g.rg2;
    r1 = min(r0 + g.rg2, m.nrep);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) branch_kernel(DevModel m, EvalOut o, SetGrid g) {
    const int32_t b = blockIdx.x;
    const int32_t idx = b % m.nbchunks;
    const int32_t r0 = (b / m.nbchunks) * g.rg1;
    const int32_t r1 = min(r0 + g.rg1, m.nrep);
    if (MODE == 0)
        branch_task(m, o, idx, r0, r1);
    else
        jt_branch_task(m, o, idx, r0, r1);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) bus_kernel(DevModel m, EvalOut o, SetGrid g) {
    __shared__ double lds[S_ROWS * kBlock];
    int32_t kind, idx, r0, r1;
    decode_phase2(g, m, blockIdx.x, kind, idx, r0, r1);
    run_task(m, o, MODE, kind, idx, r0, r1, lds);
}

// Persistent kernel: every workgroup takes work items of one phase from a
// shared queue until it is empty.  The last workgroup to leave resets the
// queue counters, so the launch can be replayed (from a graph) with no reset
// in between.
__global__ void __launch_bounds__(kBlock) batch_kernel(BatchArgs a) {
    __shared__ double lds[S_ROWS * kBlock];
    __shared__ int32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(&a.counters[0], 1);
        __syncthreads();
        const int32_t it = next;
        __syncthreads();
        if (it >= a.n_items) break;
        const BatchItem w = a.items[it];
        const BatchInst& bi = a.inst[w.inst];
        EvalOut o;
        o.x = a.X + bi.xoff;
        if (a.mode == 0) {
            o.y = a.Y ? a.Y + bi.coff : nullptr;
            o.sigma = a.sigma ? a.sigma[w.inst] : 0.0;
            o.f = a.F ? a.F + w.inst : nullptr;
            o.g = a.G ? a.G + bi.xoff : nullptr;
            o.c = a.C ? a.C + bi.coff : nullptr;
            o.J = a.J ? a.J + bi.joff : nullptr;
            o.H = a.H ? a.H + bi.hoff : nullptr;
        } else if (a.mode == 1) {
            o.y = a.Y + bi.coff;
            o.sigma = 0.0;
            o.f = o.c = o.J = o.H = nullptr;
            o.g = a.G + bi.xoff;
        } else {  // flows: X is read and its p, q entries rewritten
            o.y = nullptr;
            o.sigma = 0.0;
            o.f = o.c = o.J = o.H = nullptr;
            o.g = a.G + bi.xoff;
        }
        run_task(bi.m, o, a.mode, w.kind, w.idx, w.r0, w.r1, lds);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const int32_t done = atomicAdd(&a.counters[1], 1);
        if (done == (int32_t)gridDim.x - 1) {
            atomicExch(&a.counters[0], 0);
            atomicExch(&a.counters[1], 0);
            __threadfence();
        }
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
    g.rg2 = group_for(m.nbig + m.nwaves + m.ngchunks, m.nrep);
    g.nrg2 = (m.nrep + g.rg2 - 1) / g.rg2;
    g.n_big = any ? m.nbig * g.nrg2 : 0;
    g.n_wave = any ? m.nwaves * g.nrg2 : 0;
    if (mode == 1 && m.npg == 1 && m.nrep > 1) {
        g.gen_per_item = 1;
        g.n_gen = m.G;
    } else {
        g.gen_per_item = 0;
        g.n_gen = (any || o.f) ? m.ngchunks * g.nrg2 : 0;
    }
    return g;
}

hipError_t launch_eval_set(const DevModel& m, const EvalOut& o, hipStream_t stream) {
    const SetGrid g = plan_set(m, o, 0);
    if (g.n_branch > 0) hipLaunchKernelGGL(branch_kernel<0>, dim3(g.n_branch), dim3(kBlock), 0, stream, m, o, g);
    if (g.phase2() > 0) hipLaunchKernelGGL(bus_kernel<0>, dim3(g.phase2()), dim3(kBlock), 0, stream, m, o, g);
    return hipGetLastError();
}

hipError_t launch_jtprod(const DevModel& m, const double* x, const double* v, double* out, hipStream_t stream) {
    EvalOut o{};
    o.x = x;
    o.y = v;
    o.g = out;
    const SetGrid g = plan_set(m, o, 1);
    if (g.n_branch > 0) hipLaunchKernelGGL(branch_kernel<1>, dim3(g.n_branch), dim3(kBlock), 0, stream, m, o, g);
    if (g.phase2() > 0) hipLaunchKernelGGL(bus_kernel<1>, dim3(g.phase2()), dim3(kBlock), 0, stream, m, o, g);
    return hipGetLastError();
}

void* batch_kernel_fn() { return reinterpret_cast<void*>(&batch_kernel); }

size_t scratch_bytes(const DevModel& m) {
    const size_t parts = ((sizeof(double) * (size_t)m.ngchunks * m.npg) + 255) & ~size_t(255);
    return parts + 256 + sizeof(double) * (size_t)S_ROWS * m.nrep * m.nscr;
}

}  // namespace opf
