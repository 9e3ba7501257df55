// Internals shared by the C-ABI translation units of libopf.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "dev_model.h"
#include "eval_kernels.h"
#include "host_model.h"
#include "opf.h"

namespace opf_internal {

const std::string& last_error();
void set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx);
int set_err(int code, const char* fmt, ...);
int hip_err(hipError_t e, const char* what);

struct Allocator {
    void* (*alloc)(size_t, void*);
    void (*release)(void*, void*);
    void* ctx;
};

Allocator current_allocator();
void* dev_alloc(const Allocator& a, size_t bytes);
void dev_free(const Allocator& a, void* p);

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Host staging of many arrays packed into one device allocation.
struct Packer {
    std::vector<char> buf;
    size_t add(const void* src, size_t bytes) {
        size_t off = (buf.size() + 255) & ~size_t(255);
        buf.resize(off + std::max<size_t>(bytes, 1));
        if (src && bytes) std::memcpy(buf.data() + off, src, bytes);
        return off;
    }
    template <class T>
    size_t add(const std::vector<T>& v) {
        return add(v.data(), v.size() * sizeof(T));
    }
    size_t reserve(size_t bytes) { return add(nullptr, bytes); }
    char* at(size_t off) { return buf.data() + off; }
};

constexpr uint64_t kModelMagic = 0x4f50464d4f44454cull;  // "OPFMODEL"
constexpr uint64_t kBatchMagic = 0x4f50464241544348ull;  // "OPFBATCH"

// Offsets of the model arrays inside a packed arena.
struct ModelOffsets {
    size_t f_bus, t_bus, coef, rate2, slots, slot_coef, big_bus, adj_ptr, he, he_grp, nlo, ndist,
        hva_off, hvm_off, jbal_off, gen_ptr, gen_list, gs, bs, pd, qd, c2, c1, c0, gen_bus, ref_bus, ref_ptr,
        ref_list, outage, slots_c, tan_lim, stor_bus, stor_par, dev_bus, dev_par, st_ptr, st_list, dv_ptr, dv_list;
};

ModelOffsets pack_model(Packer& pk, const opf::HostModel& hm);
// Device descriptor of a packed model; its scratch pointers are set by
// attach_scratch.
opf::DevModel make_dev(const opf::HostModel& hm, char* base, const ModelOffsets& o);
// Point the descriptor's objective partials, ticket and half-edge records
// at `scratch` (scratch_bytes(d) bytes, the ticket zeroed).
void attach_scratch(opf::DevModel& d, char* scratch);

}  // namespace opf_internal

struct opf_model_s {
    uint64_t magic = opf_internal::kModelMagic;
    int device = 0;
    opf_internal::Allocator alloc{};
    opf::HostModel hm;
    void* arena = nullptr;
    opf::DevModel dm{};
    const int32_t *jrow = nullptr, *jcol = nullptr, *hrow = nullptr, *hcol = nullptr;
    const double *lvar = nullptr, *uvar = nullptr, *lcon = nullptr, *ucon = nullptr, *x0 = nullptr;
    const int32_t* is_ref = nullptr;
    // inverse orders for the proxy's fused loss: he_pos [2L] = position of
    // (side, branch) in the bus-ordered half-edge list he (from sides first),
    // gen_pos [G] = position of generator k in the bus-ordered gen_list
    const int32_t *he_pos = nullptr, *gen_pos = nullptr;
};

inline bool valid_model(const opf_model_s* m) { return m && m->magic == opf_internal::kModelMagic; }
