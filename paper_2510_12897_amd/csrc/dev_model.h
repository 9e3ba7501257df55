// Plain-old-data descriptors shared by the host launch code and the gfx950
// kernels: a model resident in HBM (structure-of-arrays) and one evaluation
// request.
#pragma once

#include <cstdint>

namespace opf {

// Work item kinds of one callback set.
enum TaskKind : int32_t {
    T_BUS = 0,     // a tile of consecutive buses: balance rows, Hessian bus rows
    T_BRANCH = 1,  // a block of branches: flow, angle, thermal rows, arc Hessian diagonals
    T_GEN = 2,     // a block of generators: gradient, pg Hessian diagonal, ref and ramp rows
    T_OBJ = 3      // the objective reduction (one workgroup)
};

constexpr int kBlock = 256;        // threads per workgroup, every task
constexpr int kLdsPerEdge = 8;     // doubles staged in LDS per half-edge

struct DevModel {
    int32_t N, L, G, R, T, nrep, npg, load_stride;
    int32_t ntiles, tile_cap;
    int64_t x_va, x_vm, x_pg, x_qg, x_p, x_q;
    int64_t c_ref, c_pfr, c_qfr, c_pto, c_qto, c_ang, c_balp, c_balq, c_thf, c_tht, c_ramp;
    int64_t j_ref, j_pfr, j_qfr, j_pto, j_qto, j_ang, j_balp, j_balq, j_thf, j_tht, j_ramp, jbal_rep;
    int64_t h_va, h_vm, h_pg, h_p, h_q, hva_rep, hvm_rep;
    // branches
    const int32_t* f_bus;
    const int32_t* t_bus;
    const double* coef;    // [8][L]: Gff Bff Gft Bft Gtt Btt Gtf Btf
    const double* rate2;   // [L]
    // buses
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
    const int32_t* tile_bus;  // [ntiles+1] first bus of every tile
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

// Work counts of one callback set (grid decoding of the plain launch).
struct SetGrid {
    int32_t n_bus;      // bus tiles x replicas
    int32_t n_branch;   // branch blocks x replicas
    int32_t n_gen;      // generator blocks x replicas
    int32_t n_obj;      // 0 or 1
    int32_t branch_blocks, gen_blocks;  // per replica
    int32_t total() const { return n_bus + n_branch + n_gen + n_obj; }
};

}  // namespace opf
