// Host-side model construction for the polar AC-OPF callbacks: validation,
// branch admittance terms, bus adjacency, bus tiles, the sparsity pattern and
// the bounds.  Pure C++ (no HIP); libopf uploads the result once.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "dev_model.h"
#include "opf.h"

namespace opf {

// Constraint blocks in the order the paper's Listing 3 creates them, then
// the multi-period ramp rows.  B_ANGL (the second angle-difference row) and
// B_VMAG (the voltage-magnitude row) are rows of the rectangular form only
// (Sec. III-C1); they are empty in the polar form.
// B_SOC .. B_SCMP are the storage rows (state of charge, active and
// reactive losses, thermal, complementarity), B_DRAMP / B_DINIT the device
// rows (opf_storage, opf_devices); empty without units and devices.
enum Block {
    B_REF = 0, B_PFR, B_QFR, B_PTO, B_QTO, B_ANG, B_ANGL, B_BALP, B_BALQ, B_THF, B_THT, B_VMAG, B_RAMP,
    B_SOC, B_SLP, B_SLQ, B_STH, B_SCMP, B_DRAMP, B_DINIT, B_END
};


struct Layout {
    int32_t N = 0, L = 0, G = 0, R = 0, T = 1, K = 0;
    int32_t rect = 0;   // 0: polar (va, vm); 1: rectangular (vr, vi) in the same two bus blocks
    int32_t S = 0, D = 0;  // storage units, user-extension devices
    int32_t comp = 0;      // storage complementarity rows present
    int32_t nrep = 1;   // replicas: periods or contingency copies (base + K)
    int32_t npg = 1;    // replicas of the pg block (1 when copies share pg)
    // variable blocks
    int64_t x_va = 0, x_vm = 0, x_pg = 0, x_qg = 0, x_p = 0, x_q = 0, n = 0;
    // storage blocks ps, qs, qsc, se, sc, sd and the device block u
    int64_t x_ps = 0, x_qs = 0, x_qsc = 0, x_se = 0, x_sc = 0, x_sd = 0, x_u = 0;
    // first row of each constraint block (c_blk[B_END] = m)
    int64_t c_blk[B_END + 1] = {};
    // first Jacobian entry of each block (j_blk[B_END] = nnzj)
    int64_t j_blk[B_END + 1] = {};
    int64_t jbal_rep = 0;          // entries of one replica's balance block
    // Hessian: va (vr) rows, vm (vi) rows, pg rows, p rows, q rows
    int64_t h_va = 0, h_vm = 0, h_pg = 0, h_p = 0, h_q = 0, nnzh = 0;
    // storage rows of the Hessian: ps rows [(ps, vm), (ps, ps)], qs rows
    // [(qs, vm), (qs, qs)], sd rows [(sd, sc)] (complementarity only)
    int64_t h_ps = 0, h_qs = 0, h_sd = 0;
    int64_t hva_rep = 0, hvm_rep = 0;  // entries of one replica's va / vm (vr / vi) rows

    int64_t m() const { return c_blk[B_END]; }
    int64_t nnzj() const { return j_blk[B_END]; }
};

struct HostModel {
    Layout ly;
    // branches: endpoints, 8 admittance terms (structure of arrays, term k of
    // branch l at coef[k * L + l]: Gff Bff Gft Bft Gtt Btt Gtf Btf), rate_a^2
    std::vector<int32_t> f_bus, t_bus;
    std::vector<double> coef, rate2;
    // rectangular form: tan(angmax) [L], then tan(angmin) [L]
    std::vector<double> tan_lim;
    // bus adjacency: half-edges of bus i are he[adj_ptr[i] .. adj_ptr[i+1]),
    // sorted by (neighbour bus, branch); code = branch << 1 | (bus is f_bus)
    std::vector<int32_t> adj_ptr, he, he_grp;  // he_grp: distinct-neighbour rank
    std::vector<int32_t> nlo, ndist;           // distinct neighbours below i / total
    std::vector<int32_t> hva_off, hvm_off;     // first Hessian entry of bus rows (per replica)
    std::vector<int32_t> jbal_off;             // first entry of the balance row (per replica)
    std::vector<int32_t> gen_ptr, gen_list;    // generators per bus, ascending
    std::vector<int32_t> arc_ptr, arc_list;    // arcs per bus, ascending (pattern only)
    std::vector<double> gs, bs, pd, qd;        // pd, qd: N * T for multi-period, else N
    int32_t load_stride = 0;                   // N for multi-period loads, else 0
    std::vector<double> c2, c1, c0;
    std::vector<int32_t> gen_bus;
    std::vector<int32_t> ref_bus;
    std::vector<int32_t> ref_ptr, ref_list;    // reference rows per bus, ascending
    std::vector<int32_t> is_ref;               // [N] 1 at reference buses
    std::vector<int32_t> outage;               // per replica: branch out of service or -1
    int32_t max_degree = 0;
    // storage units and devices: bus, parameters, per-bus lists (ascending)
    std::vector<int32_t> stor_bus, dev_bus;
    std::vector<double> stor_par;              // [kStorPar][S]
    std::vector<double> dev_par;               // [kDevPar][D]
    std::vector<int32_t> st_ptr, st_list, dv_ptr, dv_list;
    double stor_dt = 0.0;

    // Bus segments packed into 64-lane waves.  Each bus with at most
    // kWaveLanes - 1 incident half-edges plus generators owns a contiguous
    // segment [head, half-edges in (neighbour, branch) order, generators]
    // that never straddles a wave.  Every lane has 8 int32 fields (see
    // SlotField); output positions are relative to the replica's block.
    std::vector<int32_t> slots;                // [nwaves * kWaveLanes * 8]
    // The same lanes in the compact form the two-launch bus waves read:
    // 2 int32 per lane (kind word, index), see SlotCompact.
    std::vector<int32_t> slots_c;              // [nwaves * kWaveLanes * 2]
    int32_t nwaves = 0;
    // The 8 admittance terms of each half-edge lane's branch, in slot order
    // (zero on other lanes): a bus wave that recomputes its half-edge terms
    // reads them coalesced.
    std::vector<double> slot_coef;             // [nwaves * kWaveLanes * 8]
    std::vector<int32_t> big_bus;              // buses whose segment does not fit a wave
};

constexpr int32_t kWaveLanes = 64;

// Slot fields (int32 each): kind, ref, bus, other, jpos, h0, h1, h2.
//  kind bits [0,2): 0 idle, 1 head, 2 half-edge, 3 generator;
//       bit 2: half-edge at the branch's from bus; bit 3: first half-edge of
//       its neighbour group; bit 4: its group has parallel branches;
//       bits [8,16): segment length (head) or group length (group leader).
//  head:      bus i; jpos = first entry of i's balance Jacobian rows;
//             h0/h1/h2 = Hessian (va_i,va_i), (vm_i,va_i), (vm_i,vm_i) (-1 if absent)
//  half-edge: ref = branch, bus = i, other = neighbour; jpos = its +1 entry;
//             h0/h1/h2 = (va_i,va_k), (vm_i,va_k), (vm_i,vm_k) for the first
//             half-edge of its neighbour group, which writes the group's
//             off-diagonal entries (-1 if absent or not the group's first)
//  generator: ref = generator, bus = i; jpos = its -1 entry
//  storage unit (generator lane type, kind bit 2): ref = unit, bus = i,
//             other = the lane of its segment's head; jpos = its +1 entry
//  device (generator lane type, kind bit 4): ref = device, bus = i,
//             other = the head's lane; jpos = its entry (cp / cq)
// In the rectangular form va, vm read vr, vi: the head's h0/h2 are
// (vr_i,vr_i), (vi_i,vi_i) and h1 is absent (-1); a group's h0/h1/h2 are
// (vr_i,vr_k), (vi_i,vr_k), (vi_i,vi_k); the balance rows lead with two bus
// entries (vr_i, vi_i), so every other lane's jpos is one further on.
enum SlotKind { SK_IDLE = 0, SK_HEAD = 1, SK_EDGE = 2, SK_GEN = 3 };

// Compact slot (two launches; 8 bytes per lane instead of 32): the index is
// the bus (head) or the branch / generator (other lanes); the kind word
// holds
//   bits [0,4): as in the full kind (lane type, from side or storage unit,
//               group leader);
//   bit 4: neighbour k < i (half-edge), device (generator lane type);
//   bit 5: k > i (half-edge); bit 6: the head's bus has no branches;
//   bits [8,14): segment length - 1 (head) or group length - 1 (leader);
//   bits [14,20): lane of the segment's head in the wave;
//   bits [20,26): offset of the lane's balance Jacobian entry from the
//                 head's (0 head, 1 + q generator q, 1 + ng + arc rank,
//                 1 + ng + deg + q storage unit q, then the devices; the
//                 rectangular form adds 1 to the non-head offsets in the
//                 kernel, so that the field stays below 64);
//   bits [26,32): neighbour group of a half-edge.
// A head lane reads its bus's Hessian and Jacobian row offsets (hva_off,
// hvm_off, nlo, ndist, jbal_off); the other lanes of the segment take them
// from the head lane and form their positions from the fields above.

// Validation; returns OPF_OK or an error code with a message.
int validate(const opf_case* cs, const opf_opts* opts, std::string& err);

// Full host model; returns OPF_OK or an error code.
int build_host_model(const opf_case* cs, const opf_opts* opts, HostModel& hm, std::string& err);

// Pack the bus segments into waves (fills hm.slots, hm.nwaves, hm.big_bus).
void build_slots(HostModel& hm);

// Pattern into host buffers (any may be null).
void fill_pattern(const HostModel& hm, int32_t* jrows, int32_t* jcols, int32_t* hrows, int32_t* hcols);

// Bounds and x0 into host buffers (any may be null).
void fill_bounds(const opf_case* cs, const opf_opts* opts, const HostModel& hm, double* lvar, double* uvar,
                 double* lcon, double* ucon, double* x0);

}  // namespace opf
