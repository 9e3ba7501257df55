// gfx950 kernels for the polar AC-OPF callbacks (f, grad f, c, J, H) and
// the vector-Jacobian product J^T v.
//
// Every output entry is written exactly once by the work item that owns it,
// with no floating-point atomics; all sums run in an order fixed by the
// model, so every launch shape (plain grid, persistent batch, any replica
// grouping) gives bitwise the same results.
//
// Work items (one 64-lane wave each):
//  - waves of packed bus segments [head, half-edges, generators] (the host
//    packs them so no segment straddles a wave and precomputes every lane's
//    output positions): a half-edge lane computes its branch's second-order
//    terms for its bus, a generator lane its injection; lanes stage their
//    contributions in LDS and each head lane reduces its own segment in
//    order (a segmented reduction) into the balance rows and the bus's
//    Hessian diagonal, group leaders write the off-diagonal entries;
//  - big buses (segment wider than a wave): the same reduction over an LDS
//    tile of the bus's half-edges;
//  - branch chunks: the four flow rows, angle row and two thermal rows
//    (c, J), the arc Hessian diagonals and the arc gradient zeros;
//  - generator chunks: gradient, pg Hessian diagonal, reference and ramp
//    rows, and one objective partial per (chunk, replica); the last chunk to
//    arrive (a self-resetting ticket) sums the partials in fixed order.
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

// ------------------------------------------------------------------ waves of bus segments
struct Slot {
    int32_t kind, ref, bus, other, jpos, h0, h1, h2;
};
__device__ __forceinline__ Slot load_slot(const DevModel& m, int32_t w) {
    const int4* p = reinterpret_cast<const int4*>(m.slots) + ((size_t)w * kBlock + threadIdx.x) * 2;
    const int4 a = p[0], b = p[1];
    return Slot{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}

// LDS rows (kBlock doubles each)
enum { L_P = 0, L_Q, L_DAA, L_DMA, L_DMM, L_XAA, L_XMA, L_XMM };

__device__ void wave_task(const DevModel& m, const EvalOut& o, int32_t w, int32_t r0, int32_t r1, double* lds) {
    const int32_t lane = threadIdx.x;
    const Slot sl = load_slot(m, w);
    const int32_t type = sl.kind & 3;
    const bool from = sl.kind & 4;
    const bool leader = sl.kind & 8;
    const int32_t len = (sl.kind >> 8) & 0xff;  // segment (head) or group (leader) length
    const bool wantC = o.c != nullptr, wantH = o.H != nullptr;
    const int64_t N = m.N, L = m.L, G = m.G;
    const double* x = o.x;
    Coef k0{};
    if (type == SK_EDGE && wantH) k0 = load_coef(m, sl.ref);
    double gs = 0.0, bs = 0.0;
    if (type == SK_HEAD) {
        gs = m.gs[sl.bus];
        bs = m.bs[sl.bus];
    }
    for (int32_t r = r0; r < r1; r++) {
        double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
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
                const int64_t arc = (from ? sl.ref : sl.ref + L) + 2 * L * r;
                v[L_P] = x[m.x_p + arc];
                v[L_Q] = x[m.x_q + arc];
            }
            if (wantH) {
                const int64_t f = (from ? sl.bus : sl.other) + N * r, t = (from ? sl.other : sl.bus) + N * r;
                const double u = x[m.x_vm + f], ww = x[m.x_vm + t];
                const double th = x[m.x_va + f] - x[m.x_va + t];
                const int64_t rl = sl.ref + L * r;
                const Coef k = in_service(k0, m, sl.ref, r);
                double S, C;
                sincos(th, &S, &C);
                const Hterms h = hess_terms(k, o.y[m.c_pfr + rl], o.y[m.c_qfr + rl], o.y[m.c_pto + rl],
                                            o.y[m.c_qto + rl], u, ww, C, S);
                v[L_DAA] = h.Stt;
                v[L_DMA] = from ? h.Sut : -h.Swt;   // (vm_i, va_i)
                v[L_DMM] = from ? h.Suu : h.Sww;    // (vm_i, vm_i)
                v[L_XAA] = -h.Stt;                  // (va_f, va_t)
                v[L_XMA] = from ? -h.Sut : h.Swt;   // (vm_i, va_k)
                v[L_XMM] = h.Suw;                   // (vm_f, vm_t)
            }
        } else if (type == SK_GEN) {
            if (wantC) {
                v[L_P] = -x[m.x_pg + sl.ref + G * (m.npg > 1 ? r : 0)];
                v[L_Q] = -x[m.x_qg + sl.ref + G * r];
            }
        }
        if (wantC || wantH) {
            for (int q = 0; q < 8; q++) lds[q * kBlock + lane] = v[q];
            __syncthreads();
            if (type == SK_HEAD) {
                double sp = base_p, sq = base_q, daa = 0.0, dma = 0.0, dmm = 0.0;
                for (int32_t j = 1; j < len; j++) {  // the segment, in order
                    sp += lds[L_P * kBlock + lane + j];
                    sq += lds[L_Q * kBlock + lane + j];
                    daa += lds[L_DAA * kBlock + lane + j];
                    dma += lds[L_DMA * kBlock + lane + j];
                    dmm += lds[L_DMM * kBlock + lane + j];
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
                double xaa = v[L_XAA], xma = v[L_XMA], xmm = v[L_XMM];
                for (int32_t j = 1; j < len; j++) {  // parallel branches to one neighbour
                    xaa += lds[L_XAA * kBlock + lane + j];
                    xma += lds[L_XMA * kBlock + lane + j];
                    xmm += lds[L_XMM * kBlock + lane + j];
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

// J^T v restricted to va / vm: head lanes gather their segment.
__device__ void jt_wave_task(const DevModel& m, const EvalOut& o, int32_t w, int32_t r0, int32_t r1, double* lds) {
    const int32_t lane = threadIdx.x;
    const Slot sl = load_slot(m, w);
    const int32_t type = sl.kind & 3;
    const bool from = sl.kind & 4;
    const int32_t len = (sl.kind >> 8) & 0xff;
    const int64_t N = m.N, L = m.L;
    const double* x = o.x;
    const double* v = o.y;
    Coef k0{};
    if (type == SK_EDGE) k0 = load_coef(m, sl.ref);
    for (int32_t r = r0; r < r1; r++) {
        double ga = 0.0, gm = 0.0;
        if (type == SK_EDGE) {
            const int64_t f = (from ? sl.bus : sl.other) + N * r, t = (from ? sl.other : sl.bus) + N * r;
            const double u = x[m.x_vm + f], ww = x[m.x_vm + t];
            const double th = x[m.x_va + f] - x[m.x_va + t];
            const int64_t rl = sl.ref + L * r;
            const Coef k = in_service(k0, m, sl.ref, r);
            double S, C;
            sincos(th, &S, &C);
            const Jterms j = jt_terms(k, v[m.c_pfr + rl], v[m.c_qfr + rl], v[m.c_pto + rl], v[m.c_qto + rl], u, ww,
                                      C, S);
            const double va = v[m.c_ang + rl];
            // d th / d va_f = 1, d th / d va_t = -1; the angle row is va_f - va_t
            ga = from ? (j.Dt + va) : (-j.Dt - va);
            gm = from ? j.Du : j.Dw;
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

// ------------------------------------------------------------------ big buses (LDS tile)
__device__ void big_task(const DevModel& m, const EvalOut& o, int32_t idx, int32_t r0, int32_t r1, double* lds) {
    const int32_t b = m.big_bus[idx];
    const int32_t e0 = m.adj_ptr[b], e1 = m.adj_ptr[b + 1], deg = e1 - e0;
    const int32_t cap = m.big_cap;
    const int64_t L = m.L, N = m.N, G = m.G;
    const double* x = o.x;
    const bool wantH = o.H != nullptr, wantC = o.c != nullptr;
    const int32_t g0 = m.gen_ptr[b], ng = m.gen_ptr[b + 1] - g0;
    for (int32_t r = r0; r < r1; r++) {
        for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += kBlock) {
            const int32_t s = e - e0;
            const int32_t code = m.he[e];
            const int32_t l = code >> 1;
            const bool from = code & 1;
            if (wantC) {
                const int64_t arc = (from ? l : l + L) + 2 * L * r;
                lds[L_P * cap + s] = x[m.x_p + arc];
                lds[L_Q * cap + s] = x[m.x_q + arc];
            }
            if (wantH) {
                const int64_t f = m.f_bus[l] + N * r, t = m.t_bus[l] + N * r;
                const double u = x[m.x_vm + f], ww = x[m.x_vm + t];
                const double th = x[m.x_va + f] - x[m.x_va + t];
                const int64_t rl = l + L * r;
                const Coef k = in_service(load_coef(m, l), m, l, r);
                double S, C;
                sincos(th, &S, &C);
                const Hterms h = hess_terms(k, o.y[m.c_pfr + rl], o.y[m.c_qfr + rl], o.y[m.c_pto + rl],
                                            o.y[m.c_qto + rl], u, ww, C, S);
                lds[L_DAA * cap + s] = h.Stt;
                lds[L_DMA * cap + s] = from ? h.Sut : -h.Swt;
                lds[L_DMM * cap + s] = from ? h.Suu : h.Sww;
                lds[L_XAA * cap + s] = -h.Stt;
                lds[L_XMA * cap + s] = from ? -h.Sut : h.Swt;
                lds[L_XMM * cap + s] = h.Suw;
            }
        }
        __syncthreads();
        const int64_t bi = b + N * r;
        const double vm = x[m.x_vm + bi];
        const double gs = m.gs[b], bs = m.bs[b];
        if (wantH) {  // off-diagonal entries: one per distinct neighbour
            const int64_t hva = m.h_va + m.hva_rep * r + m.hva_off[b];
            const int64_t hvm = m.h_vm + m.hvm_rep * r + m.hvm_off[b];
            for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += kBlock) {
                const int32_t grp = m.he_grp[e];
                if (e > e0 && m.he_grp[e - 1] == grp) continue;
                const int32_t code = m.he[e], l = code >> 1;
                const int32_t k = (code & 1) ? m.t_bus[l] : m.f_bus[l];
                int32_t s = e - e0;
                double xaa = lds[L_XAA * cap + s], xma = lds[L_XMA * cap + s], xmm = lds[L_XMM * cap + s];
                for (int32_t q = e + 1; q < e1 && m.he_grp[q] == grp; q++) {
                    s = q - e0;
                    xaa += lds[L_XAA * cap + s];
                    xma += lds[L_XMA * cap + s];
                    xmm += lds[L_XMM * cap + s];
                }
                if (k < b) {
                    o.H[hva + grp] = xaa;
                    o.H[hvm + grp] = xma;
                    o.H[hvm + m.ndist[b] + 1 + grp] = xmm;
                } else {
                    o.H[hvm + grp + 1] = xma;
                }
            }
            if (threadIdx.x == 0) {
                double daa = 0.0, dma = 0.0, dmm = 0.0;
                for (int32_t s = 0; s < deg; s++) {
                    daa += lds[L_DAA * cap + s];
                    dma += lds[L_DMA * cap + s];
                    dmm += lds[L_DMM * cap + s];
                }
                const double shunt = 2.0 * gs * o.y[m.c_balp + bi] - 2.0 * bs * o.y[m.c_balq + bi];
                const int32_t nlo = m.nlo[b];
                o.H[hva + nlo] = daa;
                o.H[hvm + nlo] = dma;
                o.H[hvm + m.ndist[b] + 1 + nlo] = dmm + shunt;
            }
        }
        if (wantC && threadIdx.x == 0) {
            const int64_t ld = b + (int64_t)m.load_stride * r;
            double sp = m.pd[ld] + gs * vm * vm, sq = m.qd[ld] - bs * vm * vm;
            for (int32_t s = 0; s < deg; s++) {
                sp += lds[L_P * cap + s];
                sq += lds[L_Q * cap + s];
            }
            const int64_t pgb = m.x_pg + G * (m.npg > 1 ? r : 0), qgb = m.x_qg + G * r;
            for (int32_t q = 0; q < ng; q++) {
                sp -= x[pgb + m.gen_list[g0 + q]];
                sq -= x[qgb + m.gen_list[g0 + q]];
            }
            o.c[m.c_balp + bi] = sp;
            o.c[m.c_balq + bi] = sq;
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
        __syncthreads();
    }
}

__device__ void jt_big_task(const DevModel& m, const EvalOut& o, int32_t idx, int32_t r0, int32_t r1,
                            double* lds) {
    const int32_t b = m.big_bus[idx];
    const int32_t e0 = m.adj_ptr[b], e1 = m.adj_ptr[b + 1], deg = e1 - e0;
    const int32_t cap = m.big_cap;
    const int64_t L = m.L, N = m.N;
    const double* x = o.x;
    const double* v = o.y;
    for (int32_t r = r0; r < r1; r++) {
        for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += kBlock) {
            const int32_t s = e - e0;
            const int32_t code = m.he[e], l = code >> 1;
            const bool from = code & 1;
            const int64_t f = m.f_bus[l] + N * r, t = m.t_bus[l] + N * r;
            const double u = x[m.x_vm + f], ww = x[m.x_vm + t];
            const double th = x[m.x_va + f] - x[m.x_va + t];
            const int64_t rl = l + L * r;
            const Coef k = in_service(load_coef(m, l), m, l, r);
            double S, C;
            sincos(th, &S, &C);
            const Jterms j = jt_terms(k, v[m.c_pfr + rl], v[m.c_qfr + rl], v[m.c_pto + rl], v[m.c_qto + rl], u, ww,
                                      C, S);
            const double va = v[m.c_ang + rl];
            lds[0 * cap + s] = from ? (j.Dt + va) : (-j.Dt - va);
            lds[1 * cap + s] = from ? j.Du : j.Dw;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int64_t bi = b + N * r;
            double sa = 0.0, sm = 0.0;
            for (int32_t s = 0; s < deg; s++) {
                sa += lds[0 * cap + s];
                sm += lds[1 * cap + s];
            }
            for (int32_t q = m.ref_ptr[b]; q < m.ref_ptr[b + 1]; q++) sa += v[m.c_ref + m.ref_list[q] + (int64_t)m.R * r];
            const double vm = x[m.x_vm + bi];
            sm += 2.0 * m.gs[b] * vm * v[m.c_balp + bi] - 2.0 * m.bs[b] * vm * v[m.c_balq + bi];
            o.g[m.x_va + bi] = sa;
            o.g[m.x_vm + bi] = sm;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ branches
__device__ void branch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r0, int32_t r1) {
    const int32_t l = chunk * kBlock + (int32_t)threadIdx.x;
    if (l >= m.L) return;
    const int64_t L = m.L, N = m.N;
    const int32_t fb = m.f_bus[l], tb = m.t_bus[l];
    const bool f_lo = fb < tb;
    const bool wantCJ = o.c || o.J;
    Coef k0{};
    double rate2 = 0.0;
    if (wantCJ) {
        k0 = load_coef(m, l);
        rate2 = m.rate2[l];
    }
    const double* x = o.x;
    for (int32_t r = r0; r < r1; r++) {
        const int64_t rl = l + L * r;        // row inside a branch block
        const int64_t afr = l + 2 * L * r;   // from arc inside the p / q blocks
        const int64_t ato = afr + L;         // to arc
        if (wantCJ) {
            const double pf = x[m.x_p + afr], pt = x[m.x_p + ato];
            const double qf = x[m.x_q + afr], qt = x[m.x_q + ato];
            const Coef k = in_service(k0, m, l, r);
            const double u = x[m.x_vm + fb + N * r], w = x[m.x_vm + tb + N * r];
            const double vaf = x[m.x_va + fb + N * r], vat = x[m.x_va + tb + N * r];
            double S, C;
            sincos(vaf - vat, &S, &C);
            put_flow_row(o, m.c_pfr + rl, m.j_pfr + 5 * rl, pf, flow1(k.Gff, 0.0, k.Gft, k.Bft, u, w, C, S), f_lo);
            put_flow_row(o, m.c_qfr + rl, m.j_qfr + 5 * rl, qf, flow1(-k.Bff, 0.0, -k.Bft, k.Gft, u, w, C, S), f_lo);
            put_flow_row(o, m.c_pto + rl, m.j_pto + 5 * rl, pt, flow1(0.0, k.Gtt, k.Gtf, -k.Btf, u, w, C, S), f_lo);
            put_flow_row(o, m.c_qto + rl, m.j_qto + 5 * rl, qt, flow1(0.0, -k.Btt, -k.Btf, -k.Gtf, u, w, C, S), f_lo);
            if (o.c) {
                o.c[m.c_ang + rl] = vaf - vat;
                o.c[m.c_thf + rl] = pf * pf + qf * qf - rate2;
                o.c[m.c_tht + rl] = pt * pt + qt * qt - rate2;
            }
            if (o.J) {
                o.J[m.j_ang + 2 * rl] = f_lo ? 1.0 : -1.0;
                o.J[m.j_ang + 2 * rl + 1] = f_lo ? -1.0 : 1.0;
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
}

__device__ void jt_branch_task(const DevModel& m, const EvalOut& o, int32_t chunk, int32_t r0, int32_t r1) {
    const int32_t l = chunk * kBlock + (int32_t)threadIdx.x;
    if (l >= m.L) return;
    const int64_t L = m.L, N = m.N;
    const int32_t fb = m.f_bus[l], tb = m.t_bus[l];
    const double* x = o.x;
    const double* v = o.y;
    for (int32_t r = r0; r < r1; r++) {
        const int64_t rl = l + L * r;
        const int64_t afr = l + 2 * L * r, ato = afr + L;
        const int64_t bf = fb + N * r, bt = tb + N * r;
        const double vtf = v[m.c_thf + rl], vtt = v[m.c_tht + rl];
        // p_a sits in its flow row (+1), its bus's balance row (+1) and its
        // thermal row (2 p_a); q_a likewise
        o.g[m.x_p + afr] = v[m.c_pfr + rl] + v[m.c_balp + bf] + 2.0 * x[m.x_p + afr] * vtf;
        o.g[m.x_p + ato] = v[m.c_pto + rl] + v[m.c_balp + bt] + 2.0 * x[m.x_p + ato] * vtt;
        o.g[m.x_q + afr] = v[m.c_qfr + rl] + v[m.c_balq + bf] + 2.0 * x[m.x_q + afr] * vtf;
        o.g[m.x_q + ato] = v[m.c_qto + rl] + v[m.c_balq + bt] + 2.0 * x[m.x_q + ato] * vtt;
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

__device__ void run_task(const DevModel& m, const EvalOut& o, int32_t kind, int32_t idx, int32_t r0, int32_t r1,
                         double* lds) {
    switch (kind) {
    case T_BIG: big_task(m, o, idx, r0, r1, lds); break;
    case T_WAVE: wave_task(m, o, idx, r0, r1, lds); break;
    case T_BRANCH: branch_task(m, o, idx, r0, r1); break;
    default: gen_task(m, o, idx, r0, r1); break;
    }
}

__device__ void run_jt_task(const DevModel& m, const EvalOut& o, int32_t kind, int32_t idx, int32_t r0, int32_t r1,
                            double* lds) {
    switch (kind) {
    case T_BIG: jt_big_task(m, o, idx, r0, r1, lds); break;
    case T_WAVE: jt_wave_task(m, o, idx, r0, r1, lds); break;
    case T_BRANCH: jt_branch_task(m, o, idx, r0, r1); break;
    default: jt_gen_task(m, o, idx, r0, r1); break;
    }
}

__device__ __forceinline__ void decode_block(const SetGrid& g, const DevModel& m, int32_t b, int32_t& kind,
                                             int32_t& idx, int32_t& r0, int32_t& r1) {
    int32_t per;
    if (b < g.n_big) {
        kind = T_BIG;
        per = m.nbig;
    } else if ((b -= g.n_big) < g.n_wave) {
        kind = T_WAVE;
        per = m.nwaves;
    } else if ((b -= g.n_wave) < g.n_branch) {
        kind = T_BRANCH;
        per = m.nbchunks;
    } else {
        b -= g.n_branch;
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
    r0 = (b / per) * g.rg;
    r1 = min(r0 + g.rg, m.nrep);
}

__global__ void __launch_bounds__(kBlock) eval_set_kernel(DevModel m, EvalOut o, SetGrid grid) {
    extern __shared__ double lds[];
    int32_t kind, idx, r0, r1;
    decode_block(grid, m, blockIdx.x, kind, idx, r0, r1);
    run_task(m, o, kind, idx, r0, r1, lds);
}

__global__ void __launch_bounds__(kBlock) jtprod_kernel(DevModel m, EvalOut o, SetGrid grid) {
    extern __shared__ double lds[];
    int32_t kind, idx, r0, r1;
    decode_block(grid, m, blockIdx.x, kind, idx, r0, r1);
    run_jt_task(m, o, kind, idx, r0, r1, lds);
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
            run_task(bi.m, o, w.kind, w.idx, w.r0, w.r1, lds);
        } else {
            o.y = a.Y + bi.coff;
            o.sigma = 0.0;
            o.f = o.c = o.J = o.H = nullptr;
            o.g = a.G + bi.xoff;
            run_jt_task(bi.m, o, w.kind, w.idx, w.r0, w.r1, lds);
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

SetGrid plan_set(const DevModel& m, const EvalOut& o, int32_t mode, int32_t rg) {
    SetGrid g{};
    rg = rg < 1 ? 1 : (rg > m.nrep ? m.nrep : rg);
    g.rg = rg;
    g.nrg = (m.nrep + rg - 1) / rg;
    const bool any = mode == 1 || o.g || o.c || o.J || o.H;
    g.n_big = any ? m.nbig * g.nrg : 0;
    g.n_wave = any ? m.nwaves * g.nrg : 0;
    g.n_branch = any ? m.nbchunks * g.nrg : 0;
    if (mode == 1 && m.npg == 1 && m.nrep > 1) {
        g.gen_per_item = 1;
        g.n_gen = m.G;
    } else {
        g.gen_per_item = 0;
        g.n_gen = (any || o.f) ? m.ngchunks * g.nrg : 0;
    }
    return g;
}

size_t set_lds_bytes(const DevModel& m) {
    const size_t wave = (size_t)kLdsPerEdge * kBlock * sizeof(double);
    const size_t big = (size_t)m.big_cap * kLdsPerEdge * sizeof(double);
    return wave > big ? wave : big;
}

hipError_t launch_eval_set(const DevModel& m, const EvalOut& o, int32_t rg, hipStream_t stream) {
    const SetGrid g = plan_set(m, o, 0, rg);
    if (g.total() == 0) return hipSuccess;
    hipLaunchKernelGGL(eval_set_kernel, dim3(g.total()), dim3(kBlock), set_lds_bytes(m), stream, m, o, g);
    return hipGetLastError();
}

hipError_t launch_jtprod(const DevModel& m, const double* x, const double* v, double* out, int32_t rg,
                         hipStream_t stream) {
    EvalOut o{};
    o.x = x;
    o.y = v;
    o.g = out;
    const SetGrid g = plan_set(m, o, 1, rg);
    if (g.total() == 0) return hipSuccess;
    hipLaunchKernelGGL(jtprod_kernel, dim3(g.total()), dim3(kBlock), set_lds_bytes(m), stream, m, o, g);
    return hipGetLastError();
}

void* batch_kernel_fn() { return reinterpret_cast<void*>(&batch_kernel); }

}  // namespace opf
