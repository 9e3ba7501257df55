// Plain-old-data descriptors shared by the host launch code and the gfx950
// kernels: a model resident in HBM (structure-of-arrays) and one evaluation
// request.
#pragma once

#include <cstdint>

namespace opf {

// Work item kinds.  A callback set runs in two phases: branch and generator
// items first (they also leave each half-edge's bus-side terms in a record
// and one objective partial per generator chunk), then the bus-side items
// and the objective sum.  No item waits for another inside a launch.
enum TaskKind : int32_t {
    T_BRANCH = 0,  // phase 1: 64 branches: flow, angle, thermal rows, arc Hessian entries, half-edge records
    T_BIG = 1,     // phase 2: one bus whose segment does not fit a wave
    T_WAVE = 2,    // phase 2: 64 lanes of packed bus segments: balance rows, bus Hessian rows
    T_GEN = 3,     // phase 1: 64 generators: gradient, pg Hessian diagonal, objective partial, ref and
                   // ramp rows; J^T v: phase 2, the pg / qg entries
    T_OBJ = 4,     // phase 2 (two-launch models): the objective, summing the partials in index order
    T_STOR = 5,    // phase 1: 64 storage units: their rows, Jacobian and Hessian entries
    T_DEV = 6      // phase 1: 64 devices: their rows, gradient and objective partial
};

// Half-edge record: what the branch phase leaves for the bus phase, per
// (replica, branch, side), side 0 at the from bus, 1 at the to bus.  For the
// weighted flow-row Hessian W = sum_r -y_r hess F_r of the branch, with u the
// side's own voltage magnitude:
//   R_TT = d2W/dth2  (the bus's (va, va) term; the (va_f, va_t) entry is -R_TT)
//   R_MA = d2W/(du dva_own)  (the (vm, va) term; the (vm_own, va_other) entry is -R_MA)
//   R_MM = d2W/du2
//   R_UW = d2W/(dvm_f dvm_t)
//   R_P, R_Q = the arc's p and q (its balance-row terms)
// The J^T v phase uses the first two fields: the side's va and vm terms.
enum RecField : int32_t { R_TT = 0, R_MA, R_MM, R_UW, R_P, R_Q, kRec };
// Records are stored back to back, 48 bytes apart (16-byte aligned: three
// 16-byte loads fetch one).  Padding them to 64-byte sectors was measured
// slower, with the same three loads per lane (4 % on the 64-scenario batch)
// and with each record fetched by four cooperating lanes: the extra bytes
// written cost more than the aligned reads save.
constexpr int kRecStride = kRec;
// A set without the Hessian needs only the arc values of each half-edge:
// records [P, Q], 16 bytes apart, in the same per-side arrays.
constexpr int kRecPQ = 2;

// Storage parameters, stored [kStorPar][S] (structure of arrays).
enum StorPar : int32_t { SP_EMAX = 0, SP_CHMAX, SP_DISMAX, SP_RATING, SP_QMIN, SP_QMAX, SP_ETAC, SP_ETAD, SP_R,
                         SP_X, SP_PLOSS, SP_QLOSS, SP_E0, kStorPar };
// Device parameters the kernels read, stored [kDevPar][D].
enum DevPar : int32_t { DP_CP = 0, DP_CQ, DP_COST, kDevPar };

constexpr int kBlock = 64;          // threads per workgroup (one wave), every task
constexpr int kXcd = 8;             // XCDs; workgroups are dealt to them round-robin

struct DevModel {
    int32_t N, L, G, R, T, nrep, npg, load_stride;
    int32_t nwaves, nbig, big_cap;   // wave count, big-bus count, largest big-bus degree
    int32_t nbchunks, ngchunks;      // branch / generator chunks of kBlock
    int32_t single;                  // 1: small model; a plain callback set is one launch whose bus
                                     // items recompute their half-edge terms (batches use two)
    // block offsets and per-replica strides of x, c, J and H: 32 bits, since
    // every per-instance array stays below 2^29 elements (checked when the
    // model is created); 64-bit fields would double the scalar registers the
    // kernels spend on them
    int32_t x_va, x_vm, x_pg, x_qg, x_p, x_q;
    int32_t c_ref, c_pfr, c_qfr, c_pto, c_qto, c_ang, c_balp, c_balq, c_thf, c_tht, c_ramp;
    int32_t j_ref, j_pfr, j_qfr, j_pto, j_qto, j_ang, j_balp, j_balq, j_thf, j_tht, j_ramp, jbal_rep;
    int32_t h_va, h_vm, h_pg, h_p, h_q, hva_rep, hvm_rep;
    // branches
    const int32_t* f_bus;
    const int32_t* t_bus;
    const double* coef;    // [8][L]: Gff Bff Gft Bft Gtt Btt Gtf Btf
    const double* rate2;   // [L]
    // wave-packed bus segments: 8 int32 per lane (kind, ref, bus, other, jpos, h0, h1, h2)
    const int32_t* slots;  // [nwaves * kBlock * 8]
    const double* slot_coef;  // [nwaves * kBlock * 8] admittance terms of each half-edge lane's branch
    const int32_t* big_bus;   // [nbig]
    // bus adjacency (the big-bus path)
    const int32_t* adj_ptr;   // [N+1]
    const int32_t* he;        // [2L] branch << 1 | from-side flag, sorted by (neighbour, branch)
    const int32_t* he_grp;    // [2L] distinct-neighbour rank within the bus
    const int32_t* nlo;       // [N] distinct neighbours with a lower index
    const int32_t* ndist;     // [N] distinct neighbours
    const int32_t* hva_off;   // [N+1] first entry of the va Hessian row (one replica)
    const int32_t* hvm_off;   // [N+1] first entry of the vm Hessian row (one replica)
    const int32_t* jbal_off;  // [N+1] first entry of the balance Jacobian row (one replica)
    const int32_t* gen_ptr;   // [N+1]
    const int32_t* gen_list;  // [G] generators per bus, ascending
    const double* gs;
    const double* bs;
    const double* pd;         // [N] or [N*T]
    const double* qd;
    // generators
    const double* c2;
    const double* c1;
    const double* c0;
    const int32_t* gen_bus;   // [G]
    const int32_t* ref_bus;   // [R]
    const int32_t* ref_ptr;   // [N+1] reference rows per bus
    const int32_t* ref_list;  // [R]
    const int32_t* outage;    // [nrep] branch out of service in a replica, or -1
    // objective partials, one per (generator chunk, pg replica), and the
    // self-resetting arrival ticket of single-launch models
    double* obj_part;         // [ngchunks * npg]
    int32_t* obj_ticket;      // [1], zero between launches
    // half-edge records passed from the branch phase to the bus phase:
    // side s, replica r, branch l at rec + ((s * nrep + r) * L + l) * kRecStride
    double* rec;
    // the wave-packed bus segments again, 2 int32 per lane (kind word,
    // index): the compact form the two-launch bus waves read
    const int32_t* slots_c;   // [nwaves * kBlock * 2]
    // rectangular form (Sec. III-C1): the bus blocks at x_va, x_vm hold
    // vr, vi; each branch has a second angle row (block c_angl) and each bus
    // a voltage-magnitude row (block c_vmag).  Kept last, so that the polar
    // kernels' argument offsets do not move.
    int32_t rect;
    int32_t c_angl, c_vmag, j_angl, j_vmag;
    const double* tan_lim;    // [2][L]: tan(angmax), tan(angmin)
    // storage units and user-extension devices (S, D; their blocks of x, c,
    // J, H; per-bus lists for the wide-bus task).  Objective partials: the
    // generator chunks' (ngchunks * npg), then the device chunks'
    // (ndchunks * nrep).
    int32_t S, D, nschunks, ndchunks, comp;
    int32_t x_ps, x_qs, x_qsc, x_se, x_sc, x_sd, x_u;
    int32_t c_soc, c_slp, c_slq, c_sth, c_scmp, c_dramp, c_dinit;
    int32_t j_soc, j_slp, j_slq, j_sth, j_scmp, j_dramp, j_dinit;
    int32_t h_ps, h_qs, h_sd;
    double stor_dt;
    const int32_t* stor_bus;  // [S]
    const double* stor_par;   // [kStorPar][S]
    const int32_t* dev_bus;   // [D]
    const double* dev_par;    // [kDevPar][D]
    const int32_t* st_ptr;    // [N+1] storage units per bus, ascending
    const int32_t* st_list;
    const int32_t* dv_ptr;    // [N+1] devices per bus, ascending
    const int32_t* dv_list;
};

// Objective partials of a model: one per generator chunk and pg replica,
// then one per device chunk and replica.
#if defined(__HIP__)
__attribute__((host, device))
#endif
inline int32_t obj_slots(const DevModel& m) {
    return m.ngchunks * m.npg + m.ndchunks * m.nrep;
}

struct EvalOut {
    int32_t single;  // this launch is the single-launch shape (bus items recompute, f by ticket)
    const double* x;
    const double* y;
    double sigma;
    double* f;
    double* g;
    double* c;
    double* J;
    double* H;
};

// Work counts of one plain launch of each phase (every item covers one
// replica).  Phase-1 items are branch chunks then generator chunks;
// phase-2 items are big buses, waves, then the objective item (callback
// set) or the generator items (J^T v).
struct SetGrid {
    int32_t n_branch, n_gen1;         // phase 1 items
    int32_t n_stor, n_dev;            // phase 1 items (after the generators)
    int32_t n_big, n_wave, n_obj;     // phase 2 bus items and the objective item (0 or 1)
    int32_t n_gen2;                   // phase 2 generator items (J^T v)
    int32_t gen_per_item;             // J^T v: 0 = chunks of kBlock generators; 1 = one generator a wave
    int32_t phase1() const { return n_branch + n_gen1 + n_stor + n_dev; }
    int32_t phase2() const { return n_big + n_wave + n_obj + n_gen2; }
};

}  // namespace opf
