// Plain-old-data descriptors shared by the host launch code and the gfx950
// kernels: a model resident in HBM (structure-of-arrays) and one evaluation
// request.
#pragma once

#include <cstdint>

namespace opf {

// Work item kinds.  A callback set runs in two phases: branch items first
// (they also leave each half-edge's bus-side terms in a scratch), then the
// bus-side items.
enum TaskKind : int32_t {
    T_BRANCH = 0,  // phase 1: 64 branches: flow, angle, thermal rows, arc Hessian entries, half-edge terms
    T_BIG = 1,     // phase 2: one bus whose segment does not fit a wave
    T_WAVE = 2,    // phase 2: 64 lanes of packed bus segments: balance rows, Hessian bus diagonals
    T_GEN = 3      // phase 2: 64 generators: gradient, pg Hessian diagonal, objective, ref and ramp rows
};

// Scratch rows of the half-edge terms (one double per half-edge and replica).
enum ScratchRow : int32_t { S_P = 0, S_Q, S_DAA, S_DMA, S_DMM, S_XAA, S_XMA, S_XMM, S_ROWS };

constexpr int kBlock = 64;          // threads per workgroup (one wave), every task
constexpr int kLdsPerEdge = 8;      // doubles staged in LDS per lane / half-edge

struct DevModel {
    int32_t N, L, G, R, T, nrep, npg, load_stride;
    int32_t nwaves, nbig, big_cap;   // wave count, big-bus count, largest big-bus degree
    int32_t nscr;                    // scratch entries per replica (half-edges, wave-slot order)
    int32_t nbchunks, ngchunks;      // branch / generator chunks of kBlock
    int64_t x_va, x_vm, x_pg, x_qg, x_p, x_q;
    int64_t c_ref, c_pfr, c_qfr, c_pto, c_qto, c_ang, c_balp, c_balq, c_thf, c_tht, c_ramp;
    int64_t j_ref, j_pfr, j_qfr, j_pto, j_qto, j_ang, j_balp, j_balq, j_thf, j_tht, j_ramp, jbal_rep;
    int64_t h_va, h_vm, h_pg, h_p, h_q, hva_rep, hvm_rep;
    // branches
    const int32_t* f_bus;
    const int32_t* t_bus;
    const double* coef;    // [8][L]: Gff Bff Gft Bft Gtt Btt Gtf Btf
    const double* rate2;   // [L]
    // wave-packed bus segments: 8 int32 per lane (kind, ref, bus, other, jpos, h0, h1, h2)
    const int32_t* slots;  // [nwaves * kBlock * 8]
    const int32_t* big_bus;   // [nbig]
    const int32_t* big_scr;   // [nbig+1] first scratch entry of each big bus
    const int32_t* br_scr;    // [2][L] scratch entry of the from / to half-edge of each branch
    const int32_t* br_hx;     // [4][L] off-diagonal Hessian positions, -1 for parallel branches
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
    // objective scratch: one partial per (generator chunk, pg replica) and a
    // self-resetting arrival counter
    double* obj_part;         // [ngchunks * npg]
    int32_t* obj_ticket;      // [1]
    // half-edge terms passed from the branch phase to the bus phase:
    // row k, replica r, entry s at scr[(k * nrep + r) * nscr + s]
    double* scr;
};

struct EvalOut {
    const double* x;
    const double* y;
    double sigma;
    double* f;
    double* g;
    double* c;
    double* J;
    double* H;
};

// Work counts of one plain launch of each phase.  Phase-2 items are ordered
// big buses, waves, generator chunks; every item covers `rg` consecutive
// replicas.
struct SetGrid {
    int32_t n_branch, rg1;            // phase 1 items, replicas per item
    int32_t n_big, n_wave, n_gen;     // phase 2 items
    int32_t rg2, nrg2;                // phase 2 replicas per item, replica groups
    int32_t gen_per_item;             // 0 = chunks of kBlock generators; 1 = one generator a wave
    int32_t phase2() const { return n_big + n_wave + n_gen; }
};

}  // namespace opf
