// Launch entry points of the callback kernels (implemented in the .hip files).
#pragma once

#include <hip/hip_runtime.h>

#include "dev_model.h"

namespace opf {

// Work counts of the two launches of one model (mode 0: callback set,
// 1: J^T v).
SetGrid plan_set(const DevModel& m, const EvalOut& o, int32_t mode);

// One callback set (any subset of f, g, c, J, H) on `stream`: the branch
// phase, then the bus phase.
hipError_t launch_eval_set(const DevModel& m, const EvalOut& o, hipStream_t stream);

// out = J(x)^T v on `stream`.
hipError_t launch_jtprod(const DevModel& m, const double* x, const double* v, double* out, hipStream_t stream);

// ---- batched evaluation: one kernel per phase over a list of work items
// (persistent, or one workgroup per item).
struct BatchItem {
    int32_t inst, kind, idx, r;  // instance, task kind, entity chunk / wave / bus, replica
};

struct BatchInst {
    DevModel m;
    int64_t xoff, coff, joff, hoff;  // offsets into the concatenated arrays
};

struct BatchArgs {
    const BatchInst* inst;   // [n_inst] device
    const BatchItem* items;  // [n_items] device
    int32_t n_items;
    const double* X;
    const double* Y;
    const double* sigma;
    double *F, *G, *C, *J, *H;
    int32_t mode;            // 0 = callback set, 1 = J^T v (Y holds V, G holds OUT),
                             // 2 = arc flows (G is the X written in place)
};

// Scratch bytes a model needs per evaluation stream: objective partials,
// then the half-edge records (kRec doubles per replica, branch, side).
size_t scratch_bytes(const DevModel& m);

// The batch kernel of phase 0 (branch items) or 1 (bus items) for mode 0
// (callback set), 1 (J^T v) or 2 (flows, phase 0 only, polar only),
// persistent or flat (one workgroup per item), of the polar or the
// rectangular form, with or without storage units and devices in any
// instance (argument: BatchArgs).
void* batch_kernel_fn(int phase, int mode, bool flat, bool rect, bool ext);

// The one-launch batch kernel of callback sets (one workgroup per item:
// branch, generator, storage, device, wide-bus and wave items of every
// instance; bus lanes recompute the branch terms; objective by ticket).
void* batch_single_fn(bool rect, bool ext);

}  // namespace opf
