// gfx950 kernels for one set of polar AC-OPF callbacks (f, grad f, c, J, H).
//
// Every output entry is written exactly once by the work item that owns it,
// with no atomics, so results do not depend on scheduling:
//  - branch items (one thread per branch and replica) own the four flow rows,
//    the angle row and the two thermal rows: c, J, the p/q Hessian diagonals
//    and the zero gradient entries of the arc variables;
//  - bus tiles (a workgroup per run of consecutive buses) own the balance
//    rows and the va / vm rows of the Hessian.  One thread per half-edge
//    (bus, incident branch) computes the branch's second-order terms, stages
//    them in LDS, and the bus rows are reduced from LDS in the fixed
//    half-edge order (a segmented reduction over the bus's neighbours);
//  - generator items own the pg / qg gradient, the pg Hessian diagonal, the
//    reference-angle rows and the ramp rows;
//  - one workgroup reduces the objective in a fixed tree order.
//
// Branch flows follow the pi model (PowerModels formulation the paper uses):
//   F = alpha u^2 + beta w^2 + u w (a cos(th) + b sin(th)),
//   u = vm_f, w = vm_t, th = va_f - va_t, with (alpha, beta, a, b) per flow
//   p_fr: (Gff, 0, Gft, Bft)      q_fr: (-Bff, 0, -Bft, Gft)
//   p_to: (0, Gtt, Gtf, -Btf)     q_to: (0, -Btt, -Btf, -Gtf)
// and the flow row is c = p_arc - F.  Derivatives are written out by hand.
#include <hip/hip_runtime.h>

#include "dev_model.h"
#include "eval_kernels.h"

namespace opf {

namespace {

struct Coef {
    double Gff, Bff, Gft, Bft, Gtt, Btt, Gtf, Btf;
};

__device__ __forceinline__ Coef load_coef(const DevModel& m, int32_t l, int32_t r) {
    Coef k;
    const size_t L = (size_t)m.L;
    const double* c = m.coef;
    k.Gff = c[0 * L + l];
    k.Bff = c[1 * L + l];
    k.Gft = c[2 * L + l];
    k.Bft = c[3 * L + l];
    k.Gtt = c[4 * L + l];
    k.Btt = c[5 * L + l];
    k.Gtf = c[6 * L + l];
    k.Btf = c[7 * L + l];
    if (m.outage[r] == l) k = Coef{0, 0, 0, 0, 0, 0, 0, 0};  // branch out in this copy
    return k;
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

__device__ __forceinline__ void put_flow_row(const DevModel& m, const EvalOut& o, int64_t row, int64_t jpos,
                                             double arcval, const Flow1& fl, bool f_lo) {
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

// ------------------------------------------------------------------ branches
__device__ void branch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const int32_t l = chunk * kBlock + (int32_t)threadIdx.x;
    if (l >= m.L) return;
    const int64_t L = m.L, N = m.N;
    const int32_t f = m.f_bus[l], t = m.t_bus[l];
    const int64_t rl = l + L * r;        // row index inside a branch block
    const int64_t afr = l + 2 * L * r;   // from arc inside the p / q blocks
    const int64_t ato = afr + L;         // to arc
    const double* x = o.x;
    const double pf = x[m.x_p + afr], pt = x[m.x_p + ato];
    const double qf = x[m.x_q + afr], qt = x[m.x_q + ato];

    if (o.c || o.J) {
        const Coef k = load_coef(m, l, r);
        const double u = x[m.x_vm + f + N * r], w = x[m.x_vm + t + N * r];
        const double vaf = x[m.x_va + f + N * r], vat = x[m.x_va + t + N * r];
        double S, C;
        sincos(vaf - vat, &S, &C);
        const bool f_lo = f < t;
        put_flow_row(m, o, m.c_pfr + rl, m.j_pfr + 5 * rl, pf, flow1(k.Gff, 0.0, k.Gft, k.Bft, u, w, C, S), f_lo);
        put_flow_row(m, o, m.c_qfr + rl, m.j_qfr + 5 * rl, qf, flow1(-k.Bff, 0.0, -k.Bft, k.Gft, u, w, C, S), f_lo);
        put_flow_row(m, o, m.c_pto + rl, m.j_pto + 5 * rl, pt, flow1(0.0, k.Gtt, k.Gtf, -k.Btf, u, w, C, S), f_lo);
        put_flow_row(m, o, m.c_qto + rl, m.j_qto + 5 * rl, qt, flow1(0.0, -k.Btt, -k.Btf, -k.Gtf, u, w, C, S), f_lo);
        if (o.c) o.c[m.c_ang + rl] = vaf - vat;
        if (o.J) {
            o.J[m.j_ang + 2 * rl] = f_lo ? 1.0 : -1.0;
            o.J[m.j_ang + 2 * rl + 1] = f_lo ? -1.0 : 1.0;
        }
        const double rate2 = m.rate2[l];
        if (o.c) {
            o.c[m.c_thf + rl] = pf * pf + qf * qf - rate2;
            o.c[m.c_tht + rl] = pt * pt + qt * qt - rate2;
        }
        if (o.J) {
            o.J[m.j_thf + 2 * rl] = 2.0 * pf;
            o.J[m.j_thf + 2 * rl + 1] = 2.0 * qf;
            o.J[m.j_tht + 2 * rl] = 2.0 * pt;
            o.J[m.j_tht + 2 * rl + 1] = 2.0 * qt;
        }
    }
    if (o.H) {
        const double yf = o.y[m.c_thf + rl], yt = o.y[m.c_tht + rl];
        o.H[m.h_p + afr] = 2.0 * yf;
        o.H[m.h_p + ato] = 2.0 * yt;
        o.H[m.h_q + afr] = 2.0 * yf;
        o.H[m.h_q + ato] = 2.0 * yt;
    }
    if (o.g) {
        o.g[m.x_p + afr] = 0.0;
        o.g[m.x_p + ato] = 0.0;
        o.g[m.x_q + afr] = 0.0;
        o.g[m.x_q + ato] = 0.0;
    }
}

// ------------------------------------------------------------------ bus tiles
// LDS layout: kLdsPerEdge arrays of tile_cap doubles.
enum { S_DAA = 0, S_DMA, S_DMM, S_XAA, S_XMA, S_XMM, S_PA, S_QA };

__device__ void bus_task(const DevModel& m, const EvalOut& o, int32_t tile, int32_t r, double* lds) {
    const int32_t b0 = m.tile_bus[tile], b1 = m.tile_bus[tile + 1];
    const int32_t e0 = m.adj_ptr[b0], e1 = m.adj_ptr[b1];
    const int32_t cap = m.tile_cap;
    const int64_t L = m.L, N = m.N;
    const double* x = o.x;
    const bool wantH = o.H != nullptr;
    const bool wantC = o.c != nullptr;

    // phase 1: one thread per half-edge
    for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += kBlock) {
        const int32_t s = e - e0;
        const int32_t code = m.he[e];
        const int32_t l = code >> 1;
        const bool from = code & 1;
        if (wantC) {
            const int64_t arc = (from ? l : l + L) + 2 * L * r;
            lds[S_PA * cap + s] = x[m.x_p + arc];
            lds[S_QA * cap + s] = x[m.x_q + arc];
        }
        if (wantH) {
            const int32_t f = m.f_bus[l], t = m.t_bus[l];
            const Coef k = load_coef(m, l, r);
            const double u = x[m.x_vm + f + N * r], w = x[m.x_vm + t + N * r];
            const double th = x[m.x_va + f + N * r] - x[m.x_va + t + N * r];
            const int64_t rl = l + L * r;
            // multipliers of the four flow rows; each row is p_arc - F, so its
            // Hessian is -y * hess F, and hess F is linear in (alpha, beta, a, b)
            const double y1 = o.y[m.c_pfr + rl], y2 = o.y[m.c_qfr + rl];
            const double y3 = o.y[m.c_pto + rl], y4 = o.y[m.c_qto + rl];
            const double Wal = -(y1 * k.Gff - y2 * k.Bff);
            const double Wbe = -(y3 * k.Gtt - y4 * k.Btt);
            const double A = -(y1 * k.Gft - y2 * k.Bft + y3 * k.Gtf - y4 * k.Btf);
            const double B = -(y1 * k.Bft + y2 * k.Gft - y3 * k.Btf - y4 * k.Gtf);
            double S, C;
            sincos(th, &S, &C);
            const double K1 = A * C + B * S, K2 = B * C - A * S;
            const double Suw = K1, Stt = -u * w * K1, Sut = w * K2, Swt = u * K2;
            if (from) {  // this bus is f: u is its vm
                lds[S_DAA * cap + s] = Stt;
                lds[S_DMA * cap + s] = Sut;
                lds[S_DMM * cap + s] = 2.0 * Wal;
                lds[S_XMA * cap + s] = -Sut;   // (vm_f, va_t)
            } else {     // this bus is t: w is its vm
                lds[S_DAA * cap + s] = Stt;
                lds[S_DMA * cap + s] = -Swt;
                lds[S_DMM * cap + s] = 2.0 * Wbe;
                lds[S_XMA * cap + s] = Swt;    // (vm_t, va_f)
            }
            lds[S_XAA * cap + s] = -Stt;       // (va_f, va_t)
            lds[S_XMM * cap + s] = Suw;        // (vm_f, vm_t)
        }
    }
    __syncthreads();

    // phase 2a: off-diagonal Hessian entries, one per distinct neighbour
    if (wantH) {
        for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += kBlock) {
            const int32_t code = m.he[e];
            const int32_t l = code >> 1;
            const bool from = code & 1;
            const int32_t i = from ? m.f_bus[l] : m.t_bus[l];
            const int32_t k = from ? m.t_bus[l] : m.f_bus[l];
            const int32_t grp = m.he_grp[e];
            const int32_t ebeg = m.adj_ptr[i], eend = m.adj_ptr[i + 1];
            if (e > ebeg && m.he_grp[e - 1] == grp) continue;  // not the first of its group
            int32_t s = e - e0;
            double xaa = lds[S_XAA * cap + s], xma = lds[S_XMA * cap + s], xmm = lds[S_XMM * cap + s];
            for (int32_t q = e + 1; q < eend && m.he_grp[q] == grp; q++) {  // parallel branches
                s = q - e0;
                xaa += lds[S_XAA * cap + s];
                xma += lds[S_XMA * cap + s];
                xmm += lds[S_XMM * cap + s];
            }
            const int64_t hva = m.h_va + m.hva_rep * r + m.hva_off[i];
            const int64_t hvm = m.h_vm + m.hvm_rep * r + m.hvm_off[i];
            if (k < i) {
                o.H[hva + grp] = xaa;
                o.H[hvm + grp] = xma;
                o.H[hvm + m.ndist[i] + 1 + grp] = xmm;
            } else {
                o.H[hvm + grp + 1] = xma;
            }
        }
    }

    // phase 2b: one thread per bus
    for (int32_t i = b0 + (int32_t)threadIdx.x; i < b1; i += kBlock) {
        const int32_t s0 = m.adj_ptr[i] - e0, s1 = m.adj_ptr[i + 1] - e0;
        const int32_t deg = s1 - s0;
        const int64_t bi = i + N * r;
        const double vm = x[m.x_vm + bi];
        const double gs = m.gs[i], bs = m.bs[i];
        const int32_t g0 = m.gen_ptr[i], g1 = m.gen_ptr[i + 1];
        if (wantC) {
            const int64_t ld = i + (int64_t)m.load_stride * r;
            double sp = m.pd[ld] + gs * vm * vm;
            double sq = m.qd[ld] - bs * vm * vm;
            for (int32_t s = s0; s < s1; s++) {
                sp += lds[S_PA * cap + s];
                sq += lds[S_QA * cap + s];
            }
            const int64_t pgb = m.x_pg + (int64_t)m.G * (m.npg > 1 ? r : 0);
            const int64_t qgb = m.x_qg + (int64_t)m.G * r;
            for (int32_t q = g0; q < g1; q++) {
                const int32_t kg = m.gen_list[q];
                sp -= x[pgb + kg];
                sq -= x[qgb + kg];
            }
            o.c[m.c_balp + bi] = sp;
            o.c[m.c_balq + bi] = sq;
        }
        if (o.J) {
            double* Jp = o.J + m.j_balp + m.jbal_rep * r + m.jbal_off[i];
            double* Jq = o.J + m.j_balq + m.jbal_rep * r + m.jbal_off[i];
            Jp[0] = 2.0 * gs * vm;
            Jq[0] = -2.0 * bs * vm;
            const int32_t ng = g1 - g0;
            for (int32_t q = 1; q <= ng; q++) {
                Jp[q] = -1.0;
                Jq[q] = -1.0;
            }
            for (int32_t q = ng + 1; q <= ng + deg; q++) {
                Jp[q] = 1.0;
                Jq[q] = 1.0;
            }
        }
        if (wantH) {
            const double shunt = 2.0 * gs * o.y[m.c_balp + bi] - 2.0 * bs * o.y[m.c_balq + bi];
            const int64_t hva = m.h_va + m.hva_rep * r + m.hva_off[i];
            const int64_t hvm = m.h_vm + m.hvm_rep * r + m.hvm_off[i];
            if (deg > 0) {
                double daa = 0.0, dma = 0.0, dmm = 0.0;
                for (int32_t s = s0; s < s1; s++) {
                    daa += lds[S_DAA * cap + s];
                    dma += lds[S_DMA * cap + s];
                    dmm += lds[S_DMM * cap + s];
                }
                const int32_t nlo = m.nlo[i];
                o.H[hva + nlo] = daa;
                o.H[hvm + nlo] = dma;
                o.H[hvm + m.ndist[i] + 1 + nlo] = dmm + shunt;
            } else {
                o.H[hvm] = shunt;
            }
        }
        if (o.g) {
            o.g[m.x_va + bi] = 0.0;
            o.g[m.x_vm + bi] = 0.0;
        }
    }
}

// ------------------------------------------------------------------ generators
__device__ void gen_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const int32_t k = chunk * kBlock + (int32_t)threadIdx.x;
    const double* x = o.x;
    if (k < m.G) {
        const int64_t G = m.G;
        if (r < m.npg) {
            const int64_t col = m.x_pg + k + G * r;
            const double c2 = m.c2[k];
            if (o.g) o.g[col] = 2.0 * c2 * x[col] + m.c1[k];
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
}

// ------------------------------------------------------------------ objective
__device__ void obj_task(const DevModel& m, const EvalOut& o, double* lds) {
    if (o.f == nullptr) return;  // uniform across the workgroup: no barrier is skipped by part of it
    const int32_t G = m.G;
    const int64_t total = (int64_t)G * m.npg;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < total; j += kBlock) {
        const int32_t k = (int32_t)(j % G);
        const double pg = o.x[m.x_pg + j];
        acc += m.c2[k] * pg * pg + m.c1[k] * pg + m.c0[k];
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int32_t w = kBlock / 2; w > 0; w >>= 1) {
        if ((int32_t)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *o.f = lds[0];
}

// ------------------------------------------------------------------ J^T v
// out = J(x)^T v.  Each output entry is gathered by its owner in a fixed
// order: bus tiles own va / vm, branch items own p / q, generator items own
// pg / qg.
__device__ void jt_bus_task(const DevModel& m, const EvalOut& o, int32_t tile, int32_t r, double* lds) {
    const int32_t b0 = m.tile_bus[tile], b1 = m.tile_bus[tile + 1];
    const int32_t e0 = m.adj_ptr[b0], e1 = m.adj_ptr[b1];
    const int32_t cap = m.tile_cap;
    const int64_t L = m.L, N = m.N;
    const double* x = o.x;
    const double* v = o.y;
    for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += kBlock) {
        const int32_t s = e - e0;
        const int32_t code = m.he[e];
        const int32_t l = code >> 1;
        const bool from = code & 1;
        const int32_t f = m.f_bus[l], t = m.t_bus[l];
        const Coef k = load_coef(m, l, r);
        const double u = x[m.x_vm + f + N * r], w = x[m.x_vm + t + N * r];
        const double th = x[m.x_va + f + N * r] - x[m.x_va + t + N * r];
        const int64_t rl = l + L * r;
        const double v1 = v[m.c_pfr + rl], v2 = v[m.c_qfr + rl];
        const double v3 = v[m.c_pto + rl], v4 = v[m.c_qto + rl];
        const double va = v[m.c_ang + rl];
        // weighted flow coefficients: sum_r v_r (alpha_r, beta_r, a_r, b_r)
        const double Wal = v1 * k.Gff - v2 * k.Bff;
        const double Wbe = v3 * k.Gtt - v4 * k.Btt;
        const double A = v1 * k.Gft - v2 * k.Bft + v3 * k.Gtf - v4 * k.Btf;
        const double B = v1 * k.Bft + v2 * k.Gft - v3 * k.Btf - v4 * k.Gtf;
        double S, C;
        sincos(th, &S, &C);
        const double K1 = A * C + B * S, K2 = B * C - A * S;
        const double Ft = u * w * K2;  // sum v_r dF_r/dth
        if (from) {   // d(p - F)/dva_f = -Ft, d/dvm_f = -(2 alpha u + w K1); angle row +1
            lds[0 * cap + s] = -Ft + va;
            lds[1 * cap + s] = -(2.0 * Wal * u + w * K1);
        } else {      // d/dva_t = +Ft, d/dvm_t = -(2 beta w + u K1); angle row -1
            lds[0 * cap + s] = Ft - va;
            lds[1 * cap + s] = -(2.0 * Wbe * w + u * K1);
        }
    }
    __syncthreads();
    for (int32_t i = b0 + (int32_t)threadIdx.x; i < b1; i += kBlock) {
        const int32_t s0 = m.adj_ptr[i] - e0, s1 = m.adj_ptr[i + 1] - e0;
        const int64_t bi = i + N * r;
        double ga = 0.0, gm = 0.0;
        for (int32_t s = s0; s < s1; s++) {
            ga += lds[0 * cap + s];
            gm += lds[1 * cap + s];
        }
        for (int32_t q = m.ref_ptr[i]; q < m.ref_ptr[i + 1]; q++) ga += v[m.c_ref + m.ref_list[q] + (int64_t)m.R * r];
        const double vm = x[m.x_vm + bi];
        gm += 2.0 * m.gs[i] * vm * v[m.c_balp + bi] - 2.0 * m.bs[i] * vm * v[m.c_balq + bi];
        o.g[m.x_va + bi] = ga;
        o.g[m.x_vm + bi] = gm;
    }
}

__device__ void jt_branch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const int32_t l = chunk * kBlock + (int32_t)threadIdx.x;
    if (l >= m.L) return;
    const int64_t L = m.L, N = m.N;
    const int64_t rl = l + L * r;
    const int64_t afr = l + 2 * L * r, ato = afr + L;
    const double* x = o.x;
    const double* v = o.y;
    const int64_t bf = m.f_bus[l] + N * r, bt = m.t_bus[l] + N * r;
    const double vtf = v[m.c_thf + rl], vtt = v[m.c_tht + rl];
    // p_a appears in its flow row (+1), its bus's balance row (+1) and its
    // thermal row (2 p_a); q_a likewise
    o.g[m.x_p + afr] = v[m.c_pfr + rl] + v[m.c_balp + bf] + 2.0 * x[m.x_p + afr] * vtf;
    o.g[m.x_p + ato] = v[m.c_pto + rl] + v[m.c_balp + bt] + 2.0 * x[m.x_p + ato] * vtt;
    o.g[m.x_q + afr] = v[m.c_qfr + rl] + v[m.c_balq + bf] + 2.0 * x[m.x_q + afr] * vtf;
    o.g[m.x_q + ato] = v[m.c_qto + rl] + v[m.c_balq + bt] + 2.0 * x[m.x_q + ato] * vtt;
}

__device__ void jt_gen_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r) {
    const int32_t k = chunk * kBlock + (int32_t)threadIdx.x;
    if (k >= m.G) return;
    const int64_t G = m.G, N = m.N;
    const double* v = o.y;
    const int32_t bus = m.gen_bus[k];
    o.g[m.x_qg + k + G * r] = -v[m.c_balq + bus + N * r];
    if (r >= m.npg) return;
    double acc;
    if (m.npg == 1 && m.nrep > 1) {  // pg shared by every contingency copy
        acc = 0.0;
        for (int32_t s = 0; s < m.nrep; s++) acc -= v[m.c_balp + bus + N * s];
    } else {
        acc = -v[m.c_balp + bus + N * r];
        if (m.T > 1) {
            if (r >= 1) acc += v[m.c_ramp + k + G * (r - 1)];
            if (r + 1 < m.T) acc -= v[m.c_ramp + k + G * r];
        }
    }
    o.g[m.x_pg + k + G * r] = acc;
}

}  // namespace

__device__ void run_task(const DevModel& m, const EvalOut& o, int32_t kind, int32_t idx, int32_t rep,
                         double* lds) {
    switch (kind) {
    case T_BUS: bus_task(m, o, idx, rep, lds); break;
    case T_BRANCH: branch_task(m, o, idx, rep); break;
    case T_GEN: gen_task(m, o, idx, rep); break;
    default: obj_task(m, o, lds); break;
    }
}

__device__ void run_jt_task(const DevModel& m, const EvalOut& o, int32_t kind, int32_t idx, int32_t rep,
                            double* lds) {
    switch (kind) {
    case T_BUS: jt_bus_task(m, o, idx, rep, lds); break;
    case T_BRANCH: jt_branch_task(m, o, idx, rep); break;
    case T_GEN: jt_gen_task(m, o, idx, rep); break;
    default: break;
    }
}

__device__ __forceinline__ void decode_block(const SetGrid& grid, const DevModel& m, int32_t b, int32_t& kind,
                                             int32_t& idx, int32_t& rep) {
    if (b < grid.n_bus) {
        kind = T_BUS; idx = b % m.ntiles; rep = b / m.ntiles;
        return;
    }
    b -= grid.n_bus;
    if (b < grid.n_branch) {
        kind = T_BRANCH; idx = b % grid.branch_blocks; rep = b / grid.branch_blocks;
        return;
    }
    b -= grid.n_branch;
    if (b < grid.n_gen) {
        kind = T_GEN; idx = b % grid.gen_blocks; rep = b / grid.gen_blocks;
        return;
    }
    kind = T_OBJ; idx = 0; rep = 0;
}

__global__ void __launch_bounds__(kBlock) eval_set_kernel(DevModel m, EvalOut o, SetGrid grid) {
    extern __shared__ double lds[];
    int32_t kind, idx, rep;
    decode_block(grid, m, blockIdx.x, kind, idx, rep);
    run_task(m, o, kind, idx, rep, lds);
}

__global__ void __launch_bounds__(kBlock) jtprod_kernel(DevModel m, EvalOut o, SetGrid grid) {
    extern __shared__ double lds[];
    int32_t kind, idx, rep;
    decode_block(grid, m, blockIdx.x, kind, idx, rep);
    run_jt_task(m, o, kind, idx, rep, lds);
}

// Persistent kernel: every workgroup takes work items from a shared queue
// until it is empty.  The last workgroup to leave resets the queue counters,
// so the launch can be replayed (from a graph) with no reset in between.
__global__ void __launch_bounds__(kBlock) batch_kernel(BatchArgs a) {
    extern __shared__ double lds[];
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
            run_task(bi.m, o, w.kind, w.idx, w.rep, lds);
        } else {
            o.y = a.Y + bi.coff;
            o.g = a.G + bi.xoff;
            run_jt_task(bi.m, o, w.kind, w.idx, w.rep, lds);
        }
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

SetGrid plan_set(const DevModel& m, const EvalOut& o) {
    SetGrid g{};
    const bool any = o.g || o.c || o.J || o.H;
    g.branch_blocks = (m.L + kBlock - 1) / kBlock;
    g.gen_blocks = (std::max(m.G, m.R) + kBlock - 1) / kBlock;
    g.n_bus = any ? m.ntiles * m.nrep : 0;
    g.n_branch = any ? g.branch_blocks * m.nrep : 0;
    g.n_gen = any ? g.gen_blocks * m.nrep : 0;
    g.n_obj = o.f ? 1 : 0;
    return g;
}

size_t set_lds_bytes(const DevModel& m) {
    const size_t tile = (size_t)m.tile_cap * kLdsPerEdge * sizeof(double);
    const size_t obj = kBlock * sizeof(double);
    return tile > obj ? tile : obj;
}

hipError_t launch_eval_set(const DevModel& m, const EvalOut& o, hipStream_t stream) {
    const SetGrid g = plan_set(m, o);
    if (g.total() == 0) return hipSuccess;
    hipLaunchKernelGGL(eval_set_kernel, dim3(g.total()), dim3(kBlock), set_lds_bytes(m), stream, m, o, g);
    return hipGetLastError();
}

hipError_t launch_jtprod(const DevModel& m, const double* x, const double* v, double* out, hipStream_t stream) {
    EvalOut o{};
    o.x = x;
    o.y = v;
    o.g = out;
    SetGrid g = plan_set(m, o);
    g.n_obj = 0;
    if (g.total() == 0) return hipSuccess;
    hipLaunchKernelGGL(jtprod_kernel, dim3(g.total()), dim3(kBlock), set_lds_bytes(m), stream, m, o, g);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, int32_t grid, size_t lds_bytes, hipStream_t stream) {
    if (a.n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(kBlock), lds_bytes, stream, a);
    return hipGetLastError();
}

void* batch_kernel_fn() { return reinterpret_cast<void*>(&batch_kernel); }

}  // namespace opf
