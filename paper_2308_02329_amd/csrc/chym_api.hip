// C ABI of libchym: argument validation, device checks and dispatch.  The
// kernels live in the integrate_*.hip units (through integrate_kernel.h,
// integrate_slab.h and integrate_dispatch.hip), integrate_ell.hip,
// readout.hip, features.hip and quantize.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "chym_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(CHYM_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// The kernels are built for gfx950 only: refuse any other device up front.
int check_device() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CHYM_ENODEV, "no HIP device: %s", hipGetErrorString(e));
    static std::mutex mu;
    static int ok[64];  // 0 unknown, 1 gfx950, -1 other
    if (dev < 0 || dev >= 64) return fail(CHYM_ENODEV, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(mu);
    if (ok[dev] == 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        ok[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    }
    if (ok[dev] != 1) return fail(CHYM_ENODEV, "device %d is not gfx950", dev);
    return CHYM_OK;
}

bool finite(float v) { return isfinite(v); }

// dense storages
bool valid_jdtype(int t) { return t == CHYM_J_I8 || t == CHYM_J_F32 || t == CHYM_J_BF16 || t == CHYM_J_FP8; }
// dense or sparse rows
bool valid_jdtype_any(int t) { return valid_jdtype(t) || t == CHYM_J_ELL; }
constexpr int kEllMaxN = 4096;

int validate_problem(const chym_problem *p) {
    if (!p) return fail(CHYM_EINVAL, "problem is NULL");
    if (p->n < 1) return fail(CHYM_EINVAL, "n = %d must be >= 1", p->n);
    if (p->d < 1 || p->d > 4) return fail(CHYM_EINVAL, "d = %d must be in 1..4", p->d);
    if (!valid_jdtype_any(p->j_dtype))
        return fail(CHYM_EINVAL, "j_dtype = %d is not CHYM_J_I8, CHYM_J_F32, CHYM_J_BF16, CHYM_J_FP8 or CHYM_J_ELL",
                    p->j_dtype);
    if (!p->j) return fail(CHYM_EINVAL, "J is NULL");
    if (p->reserved != 0 || p->reserved_f != 0.0f) return fail(CHYM_EINVAL, "reserved fields must be 0");
    if (!finite(p->eps) || !finite(p->btil) || !finite(p->eta))
        return fail(CHYM_EINVAL, "eps, btil and eta must be finite");
    return CHYM_OK;
}

int validate_run(const chym_run *r) {
    if (!r) return fail(CHYM_EINVAL, "run is NULL");
    if (r->r < 1) return fail(CHYM_EINVAL, "r = %d must be >= 1", r->r);
    if (r->steps < 0) return fail(CHYM_EINVAL, "steps = %d must be >= 0", r->steps);
    if (r->start_step < 0) return fail(CHYM_EINVAL, "start_step = %d must be >= 0", r->start_step);
    if ((long long)r->start_step + r->steps > 0x7fffffffLL) return fail(CHYM_EINVAL, "start_step + steps overflows");
    if (r->precision != CHYM_PREC_F32 && r->precision != CHYM_PREC_BF16)
        return fail(CHYM_EINVAL, "precision = %d is not CHYM_PREC_F32 or CHYM_PREC_BF16", r->precision);
    if (!(r->dt > 0.0f) || !finite(r->dt)) return fail(CHYM_EINVAL, "dt must be finite and > 0");
    if (r->reserved_f != 0.0f) return fail(CHYM_EINVAL, "reserved fields must be 0");
    if (!r->pump || !r->x || !r->alpha) return fail(CHYM_EINVAL, "pump, x and alpha must not be NULL");
    return CHYM_OK;
}

// Kernel variant of a problem: 16-row tiles, state terms, coupling terms,
// and whether it runs on the register-resident kernel or, beyond its
// register budget, on the streamed-J slab kernel (which needs a workspace
// for the staged J).
struct Variant {
    int tiles, xs, js;
    bool slab;
    bool ell = false;  // sparse rows: the gather integrator
};

Variant make_variant(int n, int d, int precision, int j_dtype) {
    Variant v;
    v.tiles = (n + 15) / 16;
    v.xs = precision == CHYM_PREC_F32 ? 3 : 1;
    v.js = (precision == CHYM_PREC_F32 && j_dtype == CHYM_J_F32) ? 3 : 1;
    v.slab = v.tiles > chym::resident_tile_limit(d, v.xs, v.js);
    return v;
}

Variant variant_of(const chym_problem *p, const chym_run *r) {
    if (p->j_dtype == CHYM_J_ELL) return Variant{(p->n + 15) / 16, 1, 1, false, true};  // gather kernel, no staging
    return make_variant(p->n, p->d, r->precision, p->j_dtype);
}

size_t slab_ws_bytes(const Variant &v) { return v.slab ? chym::slab_jfrag_bytes(v.tiles, v.js) : 0; }

int default_waves_per_block() { return 4; }

chym::IntegArgs make_args(const chym_problem *prob, const chym_run *run) {
    chym::IntegArgs a;
    a.j = prob->j;
    a.pump = run->pump;
    a.x = run->x;
    a.alpha = run->alpha;
    a.n = prob->n;
    a.d = prob->d;
    a.r = run->r;
    a.steps = run->steps;
    a.start_step = run->start_step;
    a.j_dtype = prob->j_dtype;
    a.eps = prob->eps;
    a.btil = prob->btil;
    a.eta = prob->eta;
    a.dt = run->dt;
    a.kl = 0.0f;
    a.c0 = 0.0f;
    return a;
}

int check_variant(const chym_problem *prob, const chym_run *run) {
    if (prob->j_dtype == CHYM_J_ELL) {
        if (prob->n > kEllMaxN || chym::ell_replicas_per_block(prob->n, prob->d) == 0)
            return fail(CHYM_EUNSUPPORTED, "sparse couplings: n = %d must be <= %d", prob->n, kEllMaxN);
        return CHYM_OK;
    }
    const Variant v = variant_of(prob, run);
    if (v.slab && !chym::slab_variant_exists(v.tiles, prob->d, v.xs, v.js))
        return fail(CHYM_EUNSUPPORTED, "n = %d with d = %d in this precision is beyond the integrators (n <= 1024)",
                    prob->n, prob->d);
    return CHYM_OK;
}

int slab_plan_waves(const Variant &v, int d);  // block size of the streamed-J kernel from the plan table

int integrate_impl(const chym_problem *prob, const chym_run *run, hipStream_t stream, void *ws = nullptr,
                   size_t ws_bytes = 0) {
    int rc = check_variant(prob, run);
    if (rc) return rc;
    const Variant v = variant_of(prob, run);
    if (v.slab) {
        if (!ws)
            return fail(CHYM_EUNSUPPORTED, "n = %d with d = %d runs on the slab integrator, which needs a workspace "
                                           "(chym_integrate_ws / chym_solve_ws)", prob->n, prob->d);
        if (ws_bytes < slab_ws_bytes(v))
            return fail(CHYM_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, slab_ws_bytes(v));
        if ((uintptr_t)ws % 256) return fail(CHYM_EINVAL, "workspace must be 256-byte aligned");
    }
    if (run->steps == 0) return CHYM_OK;
    rc = check_device();
    if (rc) return rc;
    const chym::IntegArgs a = make_args(prob, run);
    if (prob->j_dtype == CHYM_J_ELL) {
        hipError_t e = chym::launch_integrate_ell(a, stream);
        if (e != hipSuccess) return hip_fail(e, "sparse integrate launch");
        return CHYM_OK;
    }
    if (v.slab) {
        hipError_t e = chym::launch_stage_jfrag(a, v.js, ws, stream);
        const int waves = slab_plan_waves(v, prob->d);
        if (e == hipSuccess) e = chym::launch_integrate_slab(v.tiles, prob->d, v.xs, v.js, waves, a, ws, stream);
        if (e != hipSuccess) return hip_fail(e, "slab integrate launch");
        return CHYM_OK;
    }
    bool supported = false;
    hipError_t e = chym::launch_integrate(v.tiles, prob->d, v.xs, v.js, default_waves_per_block(), a, stream,
                                          &supported);
    if (!supported) return fail(CHYM_EUNSUPPORTED, "no integrator variant for n = %d, d = %d", prob->n, prob->d);
    if (e != hipSuccess) return hip_fail(e, "integrate launch");
    return CHYM_OK;
}

// ------------------------------------------------ static scratch
// For callers that cannot allocate: the staged couplings of the streamed-J
// integrator in a file-scope device array instead of a caller workspace.
// Its size is that of the largest staging (n = 1024, i.e. 64 row tiles,
// couplings split into three bf16 terms); each GPU the library runs on holds
// its own copy until the process ends.  The staging kernels rewrite every
// byte the integrator reads, so nothing in it has to start at zero.
constexpr size_t kStaticScratchBytes = (size_t)97 << 16;  // 6.06 MiB

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[64];  // device address of `scratch` per device index

// The device address of the current device's copy of `scratch`, looked up
// once per device with that device current.  The array's name in host code
// is not a device address; only this pointer is passed to kernels.
int static_scratch(void **ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CHYM_ENODEV, "no HIP device: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return fail(CHYM_ENODEV, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(CHYM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return CHYM_OK;
}

int validate_sizes(int32_t n, int32_t d, int32_t r) {
    if (n < 1) return fail(CHYM_EINVAL, "n = %d must be >= 1", n);
    if (d < 1 || d > 4) return fail(CHYM_EINVAL, "d = %d must be in 1..4", d);
    if (r < 1) return fail(CHYM_EINVAL, "r = %d must be >= 1", r);
    return CHYM_OK;
}

int validate_energy(int32_t n, int32_t r, const void *j, int32_t j_dtype, const uint64_t *spins, int32_t *e_i32) {
    if (n < 1 || r < 1) return fail(CHYM_EINVAL, "n and r must be >= 1");
    if (n > 2048) return fail(CHYM_EUNSUPPORTED, "n = %d > 2048", n);
    if (!valid_jdtype_any(j_dtype)) return fail(CHYM_EINVAL, "bad j_dtype %d", j_dtype);
    if (!j || !spins) return fail(CHYM_EINVAL, "J and spins must not be NULL");
    if (e_i32 && j_dtype != CHYM_J_I8) return fail(CHYM_EINVAL, "int32 energy needs integer J (CHYM_J_I8)");
    return CHYM_OK;
}

int validate_hs(int32_t n, int32_t d, int32_t r, const void *j, int32_t j_dtype, const float *x) {
    int rc = validate_sizes(n, d, r);
    if (rc) return rc;
    if (n > 2048 || n * d > 8192) return fail(CHYM_EUNSUPPORTED, "hyperspin energy needs n <= 2048, n*d <= 8192");
    if (!valid_jdtype_any(j_dtype)) return fail(CHYM_EINVAL, "bad j_dtype %d", j_dtype);
    if (!j || !x) return fail(CHYM_EINVAL, "J and x must not be NULL");
    return CHYM_OK;
}


// ---------------------------------------------------------------- plans
typedef std::tuple<int, int, int, int> VariantKey;  // (tiles, d, xs, js)

struct PlanValue {
    int kind;   // chym::kKernelRegJ / kKernelLdsJ / kKernelLdsJ1 / kKernelPipe / kKernelLdsJ3 / kKernelSlab
    int waves;  // wavefronts per block
    float ms;
};

// Streamed-J variants take the slab kernel; their plans choose its block
// size.  Internal kind of such a plan.
constexpr int kKernelSlab = 100;

std::mutex g_plan_mu;
std::map<VariantKey, PlanValue> g_plan;

constexpr int kDefaultWaves = 4;
constexpr int kPersistentWaves = 4;

VariantKey key_of(const Variant &v, int d) { return std::make_tuple(v.tiles, d, v.xs, v.js); }

bool key_is_slab(const VariantKey &k) {
    return std::get<0>(k) > chym::resident_tile_limit(std::get<1>(k), std::get<2>(k), std::get<3>(k));
}

// Default block size of the slab kernel: sixteen wavefronts up to 32 row
// tiles where built (measured faster there), else eight.
int default_slab_waves(const VariantKey &k) {
    const int tiles = std::get<0>(k), d = std::get<1>(k), xs = std::get<2>(k), js = std::get<3>(k);
    return (tiles <= 32 && chym::slab_shape_exists(tiles, d, xs, js, chym::kSlabWaves16)) ? chym::kSlabWaves16
                                                                                          : chym::kSlabWaves8;
}

PlanValue plan_for(const VariantKey &k) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plan.find(k);
    if (it != g_plan.end()) return it->second;
    if (key_is_slab(k)) return PlanValue{kKernelSlab, default_slab_waves(k), 0.0f};
    return PlanValue{chym::kKernelRegJ, kDefaultWaves, 0.0f};
}

int slab_plan_waves(const Variant &v, int d) { return plan_for(key_of(v, d)).waves; }

int kind_of_code(int code) {
    switch (code) {
        case CHYM_KERNEL_LDSJ: return chym::kKernelLdsJ;
        case CHYM_KERNEL_LDSJ1: return chym::kKernelLdsJ1;
        case CHYM_KERNEL_PIPE: return chym::kKernelPipe;
        case CHYM_KERNEL_LDSJ3: return chym::kKernelLdsJ3;
        case CHYM_KERNEL_SLAB: return kKernelSlab;
        default: return chym::kKernelRegJ;
    }
}
int code_of_kind(int kind) {
    switch (kind) {
        case chym::kKernelLdsJ: return CHYM_KERNEL_LDSJ;
        case chym::kKernelLdsJ1: return CHYM_KERNEL_LDSJ1;
        case chym::kKernelPipe: return CHYM_KERNEL_PIPE;
        case chym::kKernelLdsJ3: return CHYM_KERNEL_LDSJ3;
        case kKernelSlab: return CHYM_KERNEL_SLAB;
        default: return CHYM_KERNEL_REGJ;
    }
}
bool valid_kernel_code(int code) {
    return code == CHYM_KERNEL_REGJ || code == CHYM_KERNEL_LDSJ || code == CHYM_KERNEL_LDSJ1 ||
           code == CHYM_KERNEL_PIPE || code == CHYM_KERNEL_LDSJ3 || code == CHYM_KERNEL_SLAB;
}

Variant variant_of_shape(int n, int precision, int j_dtype) {
    Variant v;
    v.tiles = (n + 15) / 16;
    v.xs = precision == CHYM_PREC_F32 ? 3 : 1;
    v.js = (precision == CHYM_PREC_F32 && j_dtype == CHYM_J_F32) ? 3 : 1;
    v.slab = false;
    return v;
}

int validate_shape(int32_t n, int32_t d, int32_t precision, int32_t j_dtype) {
    if (n < 1) return fail(CHYM_EINVAL, "n = %d must be >= 1", n);
    if (d < 1 || d > 4) return fail(CHYM_EINVAL, "d = %d must be in 1..4", d);
    if (precision != CHYM_PREC_F32 && precision != CHYM_PREC_BF16)
        return fail(CHYM_EINVAL, "precision = %d is not CHYM_PREC_F32 or CHYM_PREC_BF16", precision);
    if (!valid_jdtype(j_dtype)) return fail(CHYM_EINVAL, "bad j_dtype %d", j_dtype);
    const Variant v = variant_of_shape(n, precision, j_dtype);
    if (v.tiles > chym::resident_tile_limit(d, v.xs, v.js) && !chym::slab_variant_exists(v.tiles, d, v.xs, v.js))
        return fail(CHYM_EUNSUPPORTED, "n = %d with d = %d in this precision is beyond the integrators", n, d);
    return CHYM_OK;
}

// ---------------------------------------------------------------- batches
constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Group {
    Variant v;
    int d;
    int kind, waves;  // launch plan of this variant (resident kernels)
    int item_off, n_items;
    int blocks;
    size_t lds;  // slab kernels: LDS operand area; gather kernel: the largest block's LDS
};

struct BatchLayout {
    std::vector<Group> groups;
    std::vector<int2> items;      // (task, replica slab), grouped and sorted
    std::vector<size_t> jf_off;   // slab tasks: offset of the staged J in the workspace (else 0)
    std::vector<int> ncp;         // slab tasks: chunk count of the staging
    std::vector<int> stage_list;  // slab tasks with one coupling term, then those with three
    int n_stage1 = 0, n_stage3 = 0;
    size_t off_tasks, off_items, off_counters, off_score, off_first, off_jfp, off_ncp, off_list, off_jf, total;
    int64_t total_replicas;
    int max_nd;
    bool any_readout, any_ising, any_hs;
};

// Offsets of the batch tables in the workspace for n_tasks tasks, n_items
// work items and n_groups variant groups; the staged couplings of the
// streamed-J tasks follow at off_jf.
struct BatchTables {
    size_t off_tasks, off_items, off_counters, off_score, off_first, off_jfp, off_ncp, off_list, off_jf;
};

BatchTables batch_tables(size_t n_tasks, size_t n_items, size_t n_groups) {
    BatchTables T;
    T.off_tasks = 0;
    T.off_items = align_up(sizeof(chym::IntegArgs) * n_tasks);
    T.off_counters = T.off_items + align_up(sizeof(int2) * std::max<size_t>(1, n_items));
    T.off_score = T.off_counters + align_up(sizeof(int) * std::max<size_t>(1, n_groups));
    T.off_first = T.off_score + align_up(sizeof(chym::ScoreArgs) * n_tasks);
    T.off_jfp = T.off_first + align_up(sizeof(int64_t) * (n_tasks + 1));
    T.off_ncp = T.off_jfp + align_up(sizeof(void *) * n_tasks);
    T.off_list = T.off_ncp + align_up(sizeof(int) * n_tasks);
    T.off_jf = T.off_list + align_up(sizeof(int) * n_tasks);
    return T;
}

int validate_out(const chym_problem *prob, const chym_run *run, const chym_out *o) {
    const bool want_energy = o->e_ising || o->e_ising_f64;
    if (want_energy && !o->spins) return fail(CHYM_EINVAL, "Ising energies need the spins output");
    if (want_energy) {
        int rc = validate_energy(prob->n, run->r, prob->j, prob->j_dtype, o->spins, o->e_ising);
        if (rc) return rc;
    }
    if (o->e_hs) {
        int rc = validate_hs(prob->n, prob->d, run->r, prob->j, prob->j_dtype, run->x);
        if (rc) return rc;
    }
    return CHYM_OK;
}

int plan_layout(const chym_task *tasks, int32_t n_tasks, BatchLayout *L) {
    if (n_tasks < 1) return fail(CHYM_EINVAL, "n_tasks = %d must be >= 1", n_tasks);
    if (!tasks) return fail(CHYM_EINVAL, "tasks is NULL");
    std::map<std::tuple<int, int, int, int, int>, std::vector<int2>> by_variant;  // (slab, tiles, d, xs, js)
    for (int t = 0; t < n_tasks; ++t) {
        const chym_task &tk = tasks[t];
        int rc = validate_problem(&tk.prob);
        if (!rc) rc = validate_run(&tk.run);
        if (!rc) rc = check_variant(&tk.prob, &tk.run);
        if (!rc) rc = validate_out(&tk.prob, &tk.run, &tk.out);
        if (rc) {
            std::string m = g_err;
            return fail(rc, "task %d: %s", t, m.c_str());
        }
        const Variant v = variant_of(&tk.prob, &tk.run);
        const VariantKey key = key_of(v, tk.prob.d);
        // group key (kind, tiles, d, xs, js): kind 0 resident, 1 streamed-J, 2 sparse rows (one group per d)
        auto &lst = by_variant[v.ell ? std::make_tuple(2, 0, tk.prob.d, 0, 0)
                                     : std::make_tuple((int)v.slab, v.tiles, tk.prob.d, v.xs, v.js)];
        if (tk.run.steps == 0) continue;
        int slab = 16;
        if (v.ell) {
            slab = chym::ell_replicas_per_block(tk.prob.n, tk.prob.d);
        } else if (!v.slab) {
            const PlanValue pv = plan_for(key);
            slab = pv.kind != chym::kKernelRegJ ? 16 * pv.waves : 16;
        }
        const int slabs = (tk.run.r + slab - 1) / slab;
        for (int g = 0; g < slabs; ++g) lst.push_back(make_int2(t, g));
    }
    L->groups.clear();
    L->items.clear();
    for (auto &kv : by_variant) {
        auto &lst = kv.second;
        if (lst.empty()) continue;
        // longest first: per-item cost is proportional to the task's step count
        std::stable_sort(lst.begin(), lst.end(), [&](const int2 &a, const int2 &b) {
            return tasks[a.x].run.steps > tasks[b.x].run.steps;
        });
        Group g;
        g.v.ell = std::get<0>(kv.first) == 2;
        g.v.slab = std::get<0>(kv.first) == 1;
        g.v.tiles = std::get<1>(kv.first);
        g.d = std::get<2>(kv.first);
        g.v.xs = std::get<3>(kv.first);
        g.v.js = std::get<4>(kv.first);
        g.lds = 0;
        if (g.v.ell) {
            g.kind = -2;
            g.waves = 16;
            for (const int2 &it : lst) g.lds = std::max(g.lds, chym::ell_lds_bytes(tasks[it.x].prob.n, g.d));
        } else if (g.v.slab) {
            g.kind = -1;
            g.waves = plan_for(key_of(g.v, g.d)).waves;  // the slab kernel's block size
            g.lds = chym::slab_lds_bytes(g.v.tiles, g.d, g.v.xs);
        } else {
            const PlanValue pv = plan_for(key_of(g.v, g.d));
            g.kind = pv.kind;
            g.waves = pv.kind != chym::kKernelRegJ ? pv.waves : kPersistentWaves;
        }
        g.item_off = (int)L->items.size();
        g.n_items = (int)lst.size();
        g.blocks = 0;
        L->items.insert(L->items.end(), lst.begin(), lst.end());
        L->groups.push_back(g);
    }
    L->total_replicas = 0;
    L->max_nd = 1;
    L->any_readout = L->any_ising = L->any_hs = false;
    for (int t = 0; t < n_tasks; ++t) {
        const chym_out &o = tasks[t].out;
        L->total_replicas += tasks[t].run.r;
        L->any_readout |= (o.spins || o.extra_frac || o.diverged) != 0;
        L->any_ising |= (o.e_ising || o.e_ising_f64) != 0;
        if (o.e_hs) {
            L->any_hs = true;
            L->max_nd = std::max(L->max_nd, tasks[t].prob.n * tasks[t].prob.d);
        }
    }
    const BatchTables T = batch_tables((size_t)n_tasks, L->items.size(), L->groups.size());
    L->off_tasks = T.off_tasks;
    L->off_items = T.off_items;
    L->off_counters = T.off_counters;
    L->off_score = T.off_score;
    L->off_first = T.off_first;
    L->off_jfp = T.off_jfp;
    L->off_ncp = T.off_ncp;
    L->off_list = T.off_list;
    L->off_jf = T.off_jf;
    L->jf_off.assign(n_tasks, 0);
    L->ncp.assign(n_tasks, 0);
    L->stage_list.clear();
    std::vector<int> three;
    size_t off = L->off_jf;
    for (int t = 0; t < n_tasks; ++t) {
        const Variant v = variant_of(&tasks[t].prob, &tasks[t].run);
        if (!v.slab || tasks[t].run.steps == 0) continue;
        L->jf_off[t] = off;
        L->ncp[t] = (v.tiles + 1) / 2;
        off += align_up(slab_ws_bytes(v));
        (v.js == 3 ? three : L->stage_list).push_back(t);
    }
    L->n_stage1 = (int)L->stage_list.size();
    L->n_stage3 = (int)three.size();
    L->stage_list.insert(L->stage_list.end(), three.begin(), three.end());
    L->total = off;
    return CHYM_OK;
}

}  // namespace

struct chym_batch {
    std::vector<chym_task> tasks;
    BatchLayout layout;
    char *ws = nullptr;
    int device = -1;
    int cus = 0;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> events;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// Issues the batch on `main`: zero the work counters, one persistent kernel
// per variant group (on `branches[i]` when given, forked from and joined
// back into `main`), then the per-task scoring kernels.
int issue_batch(const chym_batch *b, hipStream_t main, const std::vector<hipStream_t> *branches,
                const std::vector<hipEvent_t> *events) {
    const BatchLayout &L = b->layout;
    const chym::IntegArgs *tasks_d = reinterpret_cast<const chym::IntegArgs *>(b->ws + L.off_tasks);
    const int2 *items_d = reinterpret_cast<const int2 *>(b->ws + L.off_items);
    int *counters = reinterpret_cast<int *>(b->ws + L.off_counters);
    hipError_t e = chym::launch_zero_counters(counters, (int)L.groups.size(), main);
    if (e != hipSuccess) return hip_fail(e, "zero counters");
    // stage the couplings of every streamed-J task: one launch per coupling-term count
    const int *list_d = reinterpret_cast<const int *>(b->ws + L.off_list);
    const int *ncp_d = reinterpret_cast<const int *>(b->ws + L.off_ncp);
    unsigned char *const *jfp_d = reinterpret_cast<unsigned char *const *>(b->ws + L.off_jfp);
    e = chym::launch_stage_batched(1, tasks_d, list_d, L.n_stage1, ncp_d, jfp_d, main);
    if (e == hipSuccess) e = chym::launch_stage_batched(3, tasks_d, list_d + L.n_stage1, L.n_stage3, ncp_d, jfp_d, main);
    if (e != hipSuccess) return hip_fail(e, "stage J");
    const bool fork = branches && L.groups.size() > 1;
    if (fork) {
        e = hipEventRecord((*events)[0], main);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    for (size_t gi = 0; gi < L.groups.size(); ++gi) {
        const Group &g = L.groups[gi];
        hipStream_t s = fork ? (*branches)[gi] : main;
        if (fork) {
            e = hipStreamWaitEvent(s, (*events)[0], 0);
            if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        }
        if (g.v.ell)
            e = chym::launch_integrate_ell_persistent(g.d, g.blocks, g.lds, tasks_d, items_d + g.item_off, g.n_items,
                                                      counters + gi, s);
        else if (g.v.slab)
            e = chym::launch_integrate_slab_persistent(
                g.v.tiles, g.d, g.v.xs, g.v.js, g.waves, g.lds, g.blocks, tasks_d, items_d + g.item_off, g.n_items,
                counters + gi, reinterpret_cast<const void *const *>(b->ws + L.off_jfp),
                reinterpret_cast<const int *>(b->ws + L.off_ncp), s);
        else
            e = chym::launch_integrate_persistent(g.v.tiles, g.d, g.v.xs, g.v.js, g.kind, g.waves, g.blocks, tasks_d,
                                                  items_d + g.item_off, g.n_items, counters + gi, s);
        if (e != hipSuccess) return hip_fail(e, "persistent integrate launch");
        if (fork) {
            e = hipEventRecord((*events)[gi + 1], s);
            if (e == hipSuccess) e = hipStreamWaitEvent(main, (*events)[gi + 1], 0);
            if (e != hipSuccess) return hip_fail(e, "join branch");
        }
    }
    if (L.any_readout || L.any_ising || L.any_hs) {
        e = chym::launch_score_batched(reinterpret_cast<const chym::ScoreArgs *>(b->ws + L.off_score),
                                       reinterpret_cast<const int64_t *>(b->ws + L.off_first), (int)b->tasks.size(),
                                       L.total_replicas, L.max_nd, L.any_readout, L.any_ising, L.any_hs, b->cus, main);
        if (e != hipSuccess) return hip_fail(e, "batched scoring launch");
    }
    return CHYM_OK;
}

void release(chym_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t ev : b->events) (void)hipEventDestroy(ev);
    for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

// ------------------------------------------------------- round-trip map
struct MapTask {
    chym::IntegArgs a;
    int tiles, xs;
};

// Validate one map problem and its run and fill the kernel arguments:
// A' = (1 - loss) [(1 - b) B - beta_b2 B S(B)] + (1 - loss) b jmag alpha (J B),  B = K(A) A.
int map_setup(const chym_map_problem *m, const chym_run *run, MapTask *t) {
    if (!m) return fail(CHYM_EINVAL, "problem is NULL");
    if (m->n < 1) return fail(CHYM_EINVAL, "n = %d must be >= 1", m->n);
    if (m->d < 1 || m->d > 4) return fail(CHYM_EINVAL, "d = %d must be in 1..4", m->d);
    if (m->j_dtype == CHYM_J_ELL) return fail(CHYM_EUNSUPPORTED, "the map form takes dense couplings");
    if (!valid_jdtype(m->j_dtype)) return fail(CHYM_EINVAL, "bad j_dtype %d", m->j_dtype);
    if (!m->j) return fail(CHYM_EINVAL, "J is NULL");
    if (m->reserved != 0 || m->reserved_f != 0.0f) return fail(CHYM_EINVAL, "reserved fields must be 0");
    if (!(m->b > 0.0f && m->b < 1.0f)) return fail(CHYM_EINVAL, "b must be in (0, 1)");
    if (!(m->loss >= 0.0f && m->loss < 1.0f)) return fail(CHYM_EINVAL, "loss must be in [0, 1)");
    if (!(m->kl > 0.0f) || !finite(m->kl)) return fail(CHYM_EINVAL, "kl must be finite and > 0");
    if (!(m->beta_b2 >= 0.0f) || !finite(m->beta_b2)) return fail(CHYM_EINVAL, "beta_b2 must be finite and >= 0");
    if (!finite(m->jmag)) return fail(CHYM_EINVAL, "jmag must be finite");
    int rc = validate_run(run);
    if (rc) return rc;
    if (run->dt != 1.0f) return fail(CHYM_EINVAL, "the map takes one round trip per step: dt must be 1");
    if (m->j_dtype == CHYM_J_F32)
        return fail(CHYM_EUNSUPPORTED, "the map form takes couplings exact in one bf16 term (I8, BF16, FP8)");
    t->tiles = (m->n + 15) / 16;
    t->xs = run->precision == CHYM_PREC_F32 ? 3 : 1;
    const int limit = std::min(chym::resident_tile_limit(m->d, t->xs, 1), chym::kMapMaxTiles);
    if (t->tiles > limit)
        return fail(CHYM_EUNSUPPORTED, "the map form runs n <= %d (n = %d, d = %d)", 16 * limit, m->n, m->d);
    chym::IntegArgs &a = t->a;
    a.j = m->j;
    a.pump = run->pump;
    a.x = run->x;
    a.alpha = run->alpha;
    a.n = m->n;
    a.d = m->d;
    a.r = run->r;
    a.steps = run->steps;
    a.start_step = run->start_step;
    a.j_dtype = m->j_dtype;
    a.dt = 1.0f;
    a.eps = (1.0f - m->loss) * m->b * m->jmag;
    a.btil = (1.0f - m->loss) * m->beta_b2;
    a.eta = 0.0f;
    a.kl = m->kl;
    a.c0 = (1.0f - m->loss) * (1.0f - m->b);
    return CHYM_OK;
}

struct MapGroup {
    int tiles, d, xs, item_off, n_items;
};

struct MapBatchLayout {
    std::vector<chym::IntegArgs> args;
    std::vector<int2> items;  // (task, 16-replica group), grouped by variant, longest task first
    std::vector<MapGroup> groups;
    size_t off_tasks, off_items, off_counters, total;
};

int map_batch_layout(const chym_map_problem *probs, const chym_run *runs, int32_t n_tasks, MapBatchLayout *L) {
    if (n_tasks < 1) return fail(CHYM_EINVAL, "n_tasks = %d must be >= 1", n_tasks);
    if (!probs || !runs) return fail(CHYM_EINVAL, "problems or runs is NULL");
    std::map<std::tuple<int, int, int>, std::vector<int2>> by_variant;  // (tiles, d, xs)
    L->args.resize(n_tasks);
    for (int t = 0; t < n_tasks; ++t) {
        MapTask mt;
        int rc = map_setup(&probs[t], &runs[t], &mt);
        if (rc) {
            std::string m = g_err;
            return fail(rc, "task %d: %s", t, m.c_str());
        }
        L->args[t] = mt.a;
        auto &lst = by_variant[std::make_tuple(mt.tiles, probs[t].d, mt.xs)];
        if (runs[t].steps == 0) continue;
        for (int g = 0; g < (runs[t].r + 15) / 16; ++g) lst.push_back(make_int2(t, g));
    }
    L->items.clear();
    L->groups.clear();
    for (auto &kv : by_variant) {
        auto &lst = kv.second;
        if (lst.empty()) continue;
        std::stable_sort(lst.begin(), lst.end(),
                         [&](const int2 &a, const int2 &b) { return runs[a.x].steps > runs[b.x].steps; });
        MapGroup g{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), (int)L->items.size(),
                   (int)lst.size()};
        L->items.insert(L->items.end(), lst.begin(), lst.end());
        L->groups.push_back(g);
    }
    L->off_tasks = 0;
    L->off_items = align_up(sizeof(chym::IntegArgs) * (size_t)n_tasks);
    L->off_counters = L->off_items + align_up(sizeof(int2) * std::max<size_t>(1, L->items.size()));
    L->total = L->off_counters + align_up(sizeof(int) * std::max<size_t>(1, L->groups.size()));
    return CHYM_OK;
}

}  // namespace

namespace {

// Validates the tasks, writes the task table and the work list into the
// caller's workspace (copies on `upload`, which is then synchronized, so the
// host tables may go away) and, when `want_graph` is set, records the launch
// sequence as a HIP graph with one branch per variant group.
int batch_build(const chym_task *tasks, int32_t n_tasks, void *workspace, size_t ws_bytes, bool want_graph,
                hipStream_t upload, chym_batch **plan) {
    if (!plan) return fail(CHYM_EINVAL, "plan is NULL");
    *plan = nullptr;
    BatchLayout L;
    int rc = plan_layout(tasks, n_tasks, &L);
    if (rc) return rc;
    if (!workspace) return fail(CHYM_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % kAlign) return fail(CHYM_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    if (ws_bytes < L.total) return fail(CHYM_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    rc = check_device();
    if (rc) return rc;
    chym_batch *b = new (std::nothrow) chym_batch;
    if (!b) return fail(CHYM_ENOMEM, "out of host memory");
    b->tasks.assign(tasks, tasks + n_tasks);
    b->layout = L;
    b->ws = static_cast<char *>(workspace);
    hipError_t e = hipGetDevice(&b->device);
    // occupancy-sized persistent grids
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    b->cus = cus;
    for (Group &g : b->layout.groups) {
        int per_cu = 0;
        if (e == hipSuccess) {
            if (g.v.ell) e = chym::ell_persistent_occupancy(g.d, g.lds, &per_cu);
            else if (g.v.slab) e = chym::slab_occupancy(g.v.tiles, g.d, g.v.xs, g.v.js, g.waves, g.lds, &per_cu);
            else e = chym::persistent_occupancy(g.v.tiles, g.d, g.v.xs, g.v.js, g.kind, g.waves, &per_cu);
        }
        const int need = (g.v.ell || g.v.slab || g.kind != chym::kKernelRegJ) ? g.n_items
                                                                              : (g.n_items + g.waves - 1) / g.waves;
        g.blocks = std::max(1, std::min(need, std::max(1, per_cu) * cus));
    }
    // task table and work list
    std::vector<chym::IntegArgs> targs(n_tasks);
    for (int t = 0; t < n_tasks; ++t) targs[t] = make_args(&tasks[t].prob, &tasks[t].run);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + L.off_tasks, targs.data(), sizeof(chym::IntegArgs) * n_tasks,
                           hipMemcpyHostToDevice, upload);
    if (e == hipSuccess && !L.items.empty())
        e = hipMemcpyAsync(b->ws + L.off_items, L.items.data(), sizeof(int2) * L.items.size(), hipMemcpyHostToDevice,
                           upload);
    std::vector<chym::ScoreArgs> sargs(n_tasks);
    std::vector<int64_t> first(n_tasks + 1, 0);
    for (int t = 0; t < n_tasks; ++t) {
        const chym_task &tk = tasks[t];
        chym::ScoreArgs &sa = sargs[t];
        sa.x = tk.run.x;
        sa.j = tk.prob.j;
        sa.spins = tk.out.spins;
        sa.e_i32 = tk.out.e_ising;
        sa.e_f64 = tk.out.e_ising_f64;
        sa.e_hs = tk.out.e_hs;
        sa.extra = tk.out.extra_frac;
        sa.diverged = tk.out.diverged;
        sa.n = tk.prob.n;
        sa.d = tk.prob.d;
        sa.r = tk.run.r;
        sa.j_dtype = tk.prob.j_dtype;
        first[t + 1] = first[t] + tk.run.r;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + L.off_score, sargs.data(), sizeof(chym::ScoreArgs) * n_tasks, hipMemcpyHostToDevice,
                           upload);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + L.off_first, first.data(), sizeof(int64_t) * (n_tasks + 1), hipMemcpyHostToDevice,
                           upload);
    std::vector<const void *> jfp(n_tasks, nullptr);
    for (int t = 0; t < n_tasks; ++t)
        if (L.jf_off[t]) jfp[t] = b->ws + L.jf_off[t];
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + L.off_jfp, jfp.data(), sizeof(void *) * n_tasks, hipMemcpyHostToDevice, upload);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + L.off_ncp, L.ncp.data(), sizeof(int) * n_tasks, hipMemcpyHostToDevice, upload);
    if (e == hipSuccess && !L.stage_list.empty())
        e = hipMemcpyAsync(b->ws + L.off_list, L.stage_list.data(), sizeof(int) * L.stage_list.size(),
                           hipMemcpyHostToDevice, upload);
    if (e == hipSuccess) e = hipStreamSynchronize(upload);  // the host tables are locals
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "batch table upload");
    }
    if (!want_graph) {
        *plan = b;
        return CHYM_OK;
    }
    // record the launch sequence as a graph with one branch per variant group
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    const size_t ng = b->layout.groups.size();
    for (size_t i = 0; e == hipSuccess && ng > 1 && i < ng; ++i) {
        hipStream_t s;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) b->side.push_back(s);
    }
    for (size_t i = 0; e == hipSuccess && ng > 1 && i < ng + 1; ++i) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->events.push_back(ev);
    }
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "batch setup");
    }
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    rc = issue_batch(b, b->cap, &b->side, &b->events);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
    b->graph = graph;
    if (rc) {
        std::string m = g_err;
        release(b);
        return fail(rc, "%s", m.c_str());
    }
    if (e2 != hipSuccess) {
        release(b);
        return hip_fail(e2, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "hipGraphInstantiate");
    }
    *plan = b;
    return CHYM_OK;
}

}  // namespace

extern "C" {

int chym_version(void) { return CHYM_VERSION; }

const char *chym_last_error(void) { return g_err.c_str(); }

int chym_integrate(const chym_problem *prob, const chym_run *run, chym_stream_t stream) {
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_run(run);
    if (rc) return rc;
    return integrate_impl(prob, run, (hipStream_t)stream);
}

int chym_map_integrate(const chym_map_problem *m, const chym_run *run, chym_stream_t stream) {
    MapTask t;
    int rc = map_setup(m, run, &t);
    if (rc) return rc;
    if (run->steps == 0) return CHYM_OK;
    rc = check_device();
    if (rc) return rc;
    bool supported = false;
    hipError_t e = chym::launch_integrate_map(t.tiles, m->d, t.xs, default_waves_per_block(), t.a,
                                              (hipStream_t)stream, &supported);
    if (!supported) return fail(CHYM_EUNSUPPORTED, "no map variant for n = %d, d = %d", m->n, m->d);
    if (e != hipSuccess) return hip_fail(e, "map integrate launch");
    return CHYM_OK;
}

int chym_map_batch_workspace_size(const chym_map_problem *probs, const chym_run *runs, int32_t n_tasks,
                                  size_t *bytes) {
    if (!bytes) return fail(CHYM_EINVAL, "bytes is NULL");
    *bytes = 0;
    MapBatchLayout L;
    int rc = map_batch_layout(probs, runs, n_tasks, &L);
    if (rc) return rc;
    *bytes = L.total;
    return CHYM_OK;
}

int chym_map_batch(const chym_map_problem *probs, const chym_run *runs, int32_t n_tasks, void *workspace,
                   size_t ws_bytes, chym_stream_t stream) {
    MapBatchLayout L;
    int rc = map_batch_layout(probs, runs, n_tasks, &L);
    if (rc) return rc;
    if (L.items.empty()) return CHYM_OK;
    if (!workspace) return fail(CHYM_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % kAlign) return fail(CHYM_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    if (ws_bytes < L.total) return fail(CHYM_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    rc = check_device();
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)stream;
    char *ws = static_cast<char *>(workspace);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // The host tables are temporaries: copy them on the stream and wait for
    // the copy before they go out of scope.
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + L.off_tasks, L.args.data(), sizeof(chym::IntegArgs) * L.args.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + L.off_items, L.items.data(), sizeof(int2) * L.items.size(), hipMemcpyHostToDevice,
                           st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int *counters = reinterpret_cast<int *>(ws + L.off_counters);
    if (e == hipSuccess) e = chym::launch_zero_counters(counters, (int)L.groups.size(), st);
    const chym::IntegArgs *tasks_d = reinterpret_cast<const chym::IntegArgs *>(ws + L.off_tasks);
    const int2 *items_d = reinterpret_cast<const int2 *>(ws + L.off_items);
    for (size_t gi = 0; gi < L.groups.size() && e == hipSuccess; ++gi) {
        const MapGroup &g = L.groups[gi];
        int per_cu = 0;
        e = chym::map_persistent_occupancy(g.tiles, g.d, g.xs, &per_cu);
        if (e != hipSuccess) break;
        const int need = (g.n_items + kPersistentWaves - 1) / kPersistentWaves;
        const int blocks = std::max(1, std::min(need, std::max(1, per_cu) * cus));
        e = chym::launch_integrate_map_persistent(g.tiles, g.d, g.xs, blocks, tasks_d, items_d + g.item_off,
                                                  g.n_items, counters + gi, st);
    }
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "map batch launch");
}

int chym_readout(int32_t n, int32_t d, int32_t r, const float *x, uint64_t *spins, double *extra_frac,
                 uint8_t *diverged, chym_stream_t stream) {
    int rc = validate_sizes(n, d, r);
    if (rc) return rc;
    if (!x) return fail(CHYM_EINVAL, "x is NULL");
    if (!spins && !extra_frac && !diverged) return CHYM_OK;
    rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_readout(n, d, r, x, spins, extra_frac, diverged, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "readout launch");
}

int chym_ising_energy(int32_t n, int32_t r, const void *j, int32_t j_dtype, const uint64_t *spins, int32_t *e_i32,
                      double *e_f64, chym_stream_t stream) {
    int rc = validate_energy(n, r, j, j_dtype, spins, e_i32);
    if (rc) return rc;
    if (!e_i32 && !e_f64) return CHYM_OK;
    rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_ising_energy(n, r, j, j_dtype, spins, e_i32, e_f64, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "ising energy launch");
}

int chym_hs_energy(int32_t n, int32_t d, int32_t r, const void *j, int32_t j_dtype, const float *x, double *e_hs,
                   chym_stream_t stream) {
    int rc = validate_hs(n, d, r, j, j_dtype, x);
    if (rc) return rc;
    if (!e_hs) return CHYM_OK;
    rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_hs_energy(n, d, r, j, j_dtype, x, e_hs, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "hyperspin energy launch");
}

int chym_solve_ws(const chym_problem *prob, const chym_run *run, int32_t ss_step, double *e_hs_ss,
                  const chym_out *out, void *workspace, size_t ws_bytes, chym_stream_t stream) {
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_run(run);
    if (rc) return rc;
    if (ss_step < 0) return fail(CHYM_EINVAL, "ss_step = %d must be >= 0", ss_step);
    const bool want_ss = e_hs_ss && ss_step > 0 && ss_step < run->steps;
    chym_out o;
    memset(&o, 0, sizeof o);
    if (out) o = *out;
    const bool want_energy = o.e_ising || o.e_ising_f64;
    if (want_energy && !o.spins) return fail(CHYM_EINVAL, "Ising energies need the spins output");
    if (want_energy) {
        rc = validate_energy(prob->n, run->r, prob->j, prob->j_dtype, o.spins, o.e_ising);
        if (rc) return rc;
    }
    if (want_ss || o.e_hs) {
        rc = validate_hs(prob->n, prob->d, run->r, prob->j, prob->j_dtype, run->x);
        if (rc) return rc;
    }
    rc = check_variant(prob, run);
    if (rc) return rc;
    const Variant v = variant_of(prob, run);
    if (v.slab && !workspace)
        return fail(CHYM_EUNSUPPORTED, "n = %d with d = %d runs on the slab integrator, which needs a workspace "
                                       "(chym_solve_ws)", prob->n, prob->d);
    if (v.slab && ws_bytes < slab_ws_bytes(v))
        return fail(CHYM_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, slab_ws_bytes(v));
    rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (want_ss) {
        chym_run a = *run;
        a.steps = ss_step;
        rc = integrate_impl(prob, &a, st, workspace, ws_bytes);
        if (rc) return rc;
        hipError_t e = chym::launch_hs_energy(prob->n, prob->d, run->r, prob->j, prob->j_dtype, run->x, e_hs_ss, st);
        if (e != hipSuccess) return hip_fail(e, "hyperspin energy launch");
        a.start_step = run->start_step + ss_step;
        a.steps = run->steps - ss_step;
        rc = integrate_impl(prob, &a, st, workspace, ws_bytes);
        if (rc) return rc;
    } else {
        rc = integrate_impl(prob, run, st, workspace, ws_bytes);
        if (rc) return rc;
    }
    hipError_t e;
    if (o.spins || o.extra_frac || o.diverged) {
        e = chym::launch_readout(prob->n, prob->d, run->r, run->x, o.spins, o.extra_frac, o.diverged, st);
        if (e != hipSuccess) return hip_fail(e, "readout launch");
    }
    if (want_energy) {
        e = chym::launch_ising_energy(prob->n, run->r, prob->j, prob->j_dtype, o.spins, o.e_ising, o.e_ising_f64, st);
        if (e != hipSuccess) return hip_fail(e, "ising energy launch");
    }
    if (o.e_hs) {
        e = chym::launch_hs_energy(prob->n, prob->d, run->r, prob->j, prob->j_dtype, run->x, o.e_hs, st);
        if (e != hipSuccess) return hip_fail(e, "hyperspin energy launch");
    }
    return CHYM_OK;
}

int chym_solve(const chym_problem *prob, const chym_run *run, int32_t ss_step, double *e_hs_ss,
               const chym_out *out, chym_stream_t stream) {
    return chym_solve_ws(prob, run, ss_step, e_hs_ss, out, nullptr, 0, stream);
}

int chym_integrate_workspace_size(const chym_problem *prob, const chym_run *run, size_t *bytes) {
    if (!bytes) return fail(CHYM_EINVAL, "bytes is NULL");
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_run(run);
    if (rc) return rc;
    rc = check_variant(prob, run);
    if (rc) return rc;
    *bytes = slab_ws_bytes(variant_of(prob, run));
    return CHYM_OK;
}

int chym_integrate_noalloc(const chym_problem *prob, const chym_run *run, chym_stream_t stream) {
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_run(run);
    if (rc) return rc;
    rc = check_variant(prob, run);
    if (rc) return rc;
    const size_t need = slab_ws_bytes(variant_of(prob, run));
    if (need == 0) return integrate_impl(prob, run, (hipStream_t)stream);  // no staging: nothing to hold
    if (need > kStaticScratchBytes)
        return fail(CHYM_EUNSUPPORTED, "n = %d with d = %d needs %zu bytes of staging; the static scratch holds %zu",
                    prob->n, prob->d, need, kStaticScratchBytes);
    void *ws = nullptr;
    rc = static_scratch(&ws);
    if (rc) return rc;
    return integrate_impl(prob, run, (hipStream_t)stream, ws, kStaticScratchBytes);
}

int chym_integrate_ws(const chym_problem *prob, const chym_run *run, void *workspace, size_t ws_bytes,
                      chym_stream_t stream) {
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_run(run);
    if (rc) return rc;
    return integrate_impl(prob, run, (hipStream_t)stream, workspace, ws_bytes);
}

int chym_batch_workspace_size(const chym_task *tasks, int32_t n_tasks, size_t *bytes) {
    if (!bytes) return fail(CHYM_EINVAL, "bytes is NULL");
    BatchLayout L;
    int rc = plan_layout(tasks, n_tasks, &L);
    if (rc) return rc;
    *bytes = L.total;
    return CHYM_OK;
}

int chym_batch_create(const chym_task *tasks, int32_t n_tasks, void *workspace, size_t ws_bytes,
                      chym_batch **plan) {
    return batch_build(tasks, n_tasks, workspace, ws_bytes, true, nullptr, plan);
}

int chym_solve_batched(const chym_task *tasks, int32_t n_tasks, void *workspace, size_t ws_bytes,
                       chym_stream_t stream) {
    chym_batch *b = nullptr;
    int rc = batch_build(tasks, n_tasks, workspace, ws_bytes, false, (hipStream_t)stream, &b);
    if (rc) return rc;
    rc = issue_batch(b, (hipStream_t)stream, nullptr, nullptr);
    // the plan is host data only; the queued kernels hold their arguments
    release(b);
    return rc;
}

int chym_batch_launch(const chym_batch *plan, chym_stream_t stream) {
    if (!plan || !plan->exec) return fail(CHYM_EINVAL, "plan is NULL");
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "hipGraphLaunch");
}

int chym_batch_launch_nograph(const chym_batch *plan, chym_stream_t stream) {
    if (!plan) return fail(CHYM_EINVAL, "plan is NULL");
    return issue_batch(plan, (hipStream_t)stream, nullptr, nullptr);
}

int chym_batch_destroy(chym_batch *plan) {
    if (!plan) return CHYM_OK;
    hipError_t e = hipDeviceSynchronize();
    release(plan);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "hipDeviceSynchronize");
}

// ------------------------------------------------------------------ plans
int chym_plan_set(const chym_plan_entry *e) {
    if (!e) return fail(CHYM_EINVAL, "entry is NULL");
    int rc = validate_shape(e->n, e->d, e->precision, e->j_dtype);
    if (rc) return rc;
    if (e->reserved != 0.0f) return fail(CHYM_EINVAL, "reserved fields must be 0");
    const VariantKey k = key_of(variant_of_shape(e->n, e->precision, e->j_dtype), e->d);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (e->kernel == CHYM_KERNEL_AUTO) {
        g_plan.erase(k);
        return CHYM_OK;
    }
    if (!valid_kernel_code(e->kernel)) return fail(CHYM_EINVAL, "kernel = %d is not a CHYM_KERNEL_* value", e->kernel);
    if (key_is_slab(k) != (e->kernel == CHYM_KERNEL_SLAB))
        return fail(CHYM_EUNSUPPORTED, "n = %d, d = %d in this form runs on the %s kernel: kernel must %s CHYM_KERNEL_SLAB",
                    e->n, e->d, key_is_slab(k) ? "streamed-J" : "register-resident", key_is_slab(k) ? "be" : "not be");
    if (e->kernel == CHYM_KERNEL_SLAB) {
        if (e->waves != chym::kSlabWaves8 && e->waves != chym::kSlabWaves16)
            return fail(CHYM_EINVAL, "waves = %d must be 8 or 16 for the streamed-J kernel", e->waves);
        if (!chym::slab_shape_exists(std::get<0>(k), e->d, std::get<2>(k), std::get<3>(k), e->waves))
            return fail(CHYM_EUNSUPPORTED, "no streamed-J block of %d wavefronts for n = %d, d = %d in this form",
                        e->waves, e->n, e->d);
    } else {
        if (e->waves < 1 || e->waves > 4) return fail(CHYM_EINVAL, "waves = %d must be in 1..4", e->waves);
        if (!chym::persistent_kind_exists(std::get<0>(k), e->d, std::get<2>(k), std::get<3>(k), kind_of_code(e->kernel)))
            return fail(CHYM_EUNSUPPORTED, "kernel = %d is not built for n = %d, d = %d in this form", e->kernel, e->n,
                        e->d);
    }
    g_plan[k] = PlanValue{kind_of_code(e->kernel), e->waves, e->ms};
    return CHYM_OK;
}

int chym_plan_get(int32_t n, int32_t d, int32_t precision, int32_t j_dtype, chym_plan_entry *e) {
    if (!e) return fail(CHYM_EINVAL, "entry is NULL");
    int rc = validate_shape(n, d, precision, j_dtype);
    if (rc) return rc;
    const PlanValue pv = plan_for(key_of(variant_of_shape(n, precision, j_dtype), d));
    e->n = n;
    e->d = d;
    e->precision = precision;
    e->j_dtype = j_dtype;
    e->kernel = code_of_kind(pv.kind);
    e->waves = pv.waves;
    e->ms = pv.ms;
    e->reserved = 0.0f;
    return CHYM_OK;
}

namespace {
struct ProbeLayout {
    size_t off_j, off_pump, off_x, off_alpha, off_batch, total, batch_bytes;
};

ProbeLayout probe_layout(int n, int d, int r, int steps) {
    ProbeLayout L;
    L.off_j = 0;
    L.off_pump = align_up((size_t)n * n * 4);
    L.off_x = L.off_pump + align_up((size_t)r * 4);
    L.off_alpha = L.off_x + align_up((size_t)n * r * d * 4);
    L.off_batch = L.off_alpha + align_up((size_t)steps * d * 4);
    // batch workspace of one task: its work list is largest with 16-replica
    // items; the staged couplings of a streamed-J task follow the tables
    // (sized for three coupling terms, the most any form stages)
    L.batch_bytes = batch_tables(1, (size_t)((r + 15) / 16), 1).off_jf + align_up(chym::slab_jfrag_bytes((n + 15) / 16, 3));
    L.total = L.off_batch + L.batch_bytes;
    return L;
}
}  // namespace

int chym_plan_autotune_workspace_size(int32_t n, int32_t d, int32_t replicas, int32_t steps, size_t *bytes) {
    if (!bytes) return fail(CHYM_EINVAL, "bytes is NULL");
    if (n < 1 || d < 1 || d > 4 || replicas < 1 || steps < 1) return fail(CHYM_EINVAL, "bad probe shape");
    *bytes = probe_layout(n, d, replicas, steps).total;
    return CHYM_OK;
}

constexpr int kTimedReps = 3;  // timed runs per autotune candidate (after one warm-up); the fastest counts

int chym_plan_autotune(int32_t n, int32_t d, int32_t precision, int32_t j_dtype, int32_t replicas, int32_t steps,
                       void *workspace, size_t ws_bytes, chym_plan_entry *best, chym_plan_entry *cand,
                       int32_t max_cand, int32_t *n_cand, chym_stream_t stream) {
    int rc = validate_shape(n, d, precision, j_dtype);
    if (rc) return rc;
    if (replicas < 1 || steps < 1) return fail(CHYM_EINVAL, "replicas and steps must be >= 1");
    if (!workspace || !best) return fail(CHYM_EINVAL, "workspace and best must not be NULL");
    if ((uintptr_t)workspace % kAlign) return fail(CHYM_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    const ProbeLayout L = probe_layout(n, d, replicas, steps);
    if (ws_bytes < L.total) return fail(CHYM_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *ws = static_cast<char *>(workspace);
    // the integrator variant depends on J's storage only through its term count: probe with
    // float32 J when it is split, else with +-1 int8 J
    const int probe_jt = (j_dtype == CHYM_J_F32) ? CHYM_J_F32 : CHYM_J_I8;
    hipError_t e = chym::launch_fill_probe(ws + L.off_j, probe_jt, n, reinterpret_cast<float *>(ws + L.off_pump),
                                           replicas, reinterpret_cast<float *>(ws + L.off_alpha), steps * d, st);
    if (e != hipSuccess) return hip_fail(e, "probe fill");
    chym_task task;
    memset(&task, 0, sizeof task);
    task.prob.n = n;
    task.prob.d = d;
    task.prob.j_dtype = probe_jt;
    task.prob.j = ws + L.off_j;
    task.prob.eps = 0.05f;
    task.prob.btil = 1.0f;
    task.prob.eta = 2e-4f;
    task.run.r = replicas;
    task.run.steps = steps;
    task.run.precision = precision;
    task.run.dt = 0.01f;
    task.run.pump = reinterpret_cast<const float *>(ws + L.off_pump);
    task.run.x = reinterpret_cast<float *>(ws + L.off_x);
    task.run.alpha = reinterpret_cast<const float *>(ws + L.off_alpha);
    const VariantKey key = key_of(variant_of_shape(n, precision, j_dtype), d);
    PlanValue saved;
    bool had;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plan.find(key);
        had = it != g_plan.end();
        if (had) saved = it->second;
    }
    const PlanValue all_cands[] = {{chym::kKernelRegJ, 4, 0.f},
                                   {chym::kKernelLdsJ, 2, 0.f},
                                   {chym::kKernelLdsJ, 4, 0.f},
                                   {chym::kKernelLdsJ1, 4, 0.f},
                                   {chym::kKernelPipe, 4, 0.f},
                                   {chym::kKernelLdsJ3, 4, 0.f},
                                   {kKernelSlab, chym::kSlabWaves8, 0.f},
                                   {kKernelSlab, chym::kSlabWaves16, 0.f}};
    PlanValue cands[sizeof(all_cands) / sizeof(all_cands[0])];
    int kCands = 0;
    const bool slab = key_is_slab(key);
    for (const PlanValue &pv : all_cands) {
        const bool ok = slab ? (pv.kind == kKernelSlab &&
                                chym::slab_shape_exists(std::get<0>(key), d, std::get<2>(key), std::get<3>(key), pv.waves))
                             : (pv.kind != kKernelSlab &&
                                chym::persistent_kind_exists(std::get<0>(key), d, std::get<2>(key), std::get<3>(key), pv.kind));
        if (ok) cands[kCands++] = pv;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    int best_i = -1;
    float best_ms = 0.0f;
    int count = 0;
    rc = CHYM_OK;
    for (int ci = 0; ci < kCands && rc == CHYM_OK; ++ci) {
        {
            std::lock_guard<std::mutex> lk(g_plan_mu);
            g_plan[key] = cands[ci];
        }
        chym_batch *plan = nullptr;
        rc = chym_batch_create(&task, 1, ws + L.off_batch, L.batch_bytes, &plan);
        if (rc) break;
        float ms = 0.0f;
        for (int rep = 0; rep < 1 + kTimedReps && rc == CHYM_OK; ++rep) {  // warm-up, then the fastest timed run
            float t = 0.0f;
            e = chym::launch_fill_state(task.run.x, (size_t)n * replicas * d, st);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            if (e == hipSuccess) rc = chym_batch_launch_nograph(plan, st);
            if (e == hipSuccess && rc == CHYM_OK) e = hipEventRecord(e1, st);
            if (e == hipSuccess && rc == CHYM_OK) e = hipEventSynchronize(e1);
            if (e == hipSuccess && rc == CHYM_OK) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) rc = hip_fail(e, "autotune timing");
            if (rep == 1 || (rep > 1 && t < ms)) ms = t;
        }
        chym_batch_destroy(plan);
        if (rc) break;
        if (cand && count < max_cand) {
            chym_plan_entry &c = cand[count];
            c.n = n;
            c.d = d;
            c.precision = precision;
            c.j_dtype = j_dtype;
            c.kernel = code_of_kind(cands[ci].kind);
            c.waves = cands[ci].waves;
            c.ms = ms;
            c.reserved = 0.0f;
        }
        ++count;
        if (best_i < 0 || ms < best_ms) {
            best_i = ci;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        if (rc != CHYM_OK || best_i < 0) {
            if (had) g_plan[key] = saved;
            else g_plan.erase(key);
        } else {
            PlanValue pv = cands[best_i];
            pv.ms = best_ms;
            g_plan[key] = pv;
        }
    }
    if (n_cand) *n_cand = std::min(count, max_cand);
    if (rc) return rc;
    return chym_plan_get(n, d, precision, j_dtype, best);
}

int chym_j_bytes(int32_t n, int32_t j_dtype, size_t *bytes) {
    if (!bytes) return fail(CHYM_EINVAL, "bytes is NULL");
    if (n < 1) return fail(CHYM_EINVAL, "n = %d must be >= 1", n);
    if (j_dtype == CHYM_J_ELL) return fail(CHYM_EINVAL, "sparse couplings take 8 w (n + 1) bytes for row width w");
    if (!valid_jdtype(j_dtype)) return fail(CHYM_EINVAL, "bad j_dtype %d", j_dtype);
    const size_t nn = (size_t)n * n;
    switch (j_dtype) {
        case CHYM_J_I8: *bytes = nn; break;
        case CHYM_J_F32: *bytes = 4 * nn; break;
        case CHYM_J_BF16: *bytes = 2 * nn; break;
        default: *bytes = nn + (size_t)n; break;
    }
    return CHYM_OK;
}

int chym_quantize_fp8(int32_t n, const float *j, uint8_t *out, chym_stream_t stream) {
    if (n < 1) return fail(CHYM_EINVAL, "n = %d must be >= 1", n);
    if (!j || !out) return fail(CHYM_EINVAL, "j and out must not be NULL");
    int rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_quantize_fp8(n, j, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "quantize launch");
    return CHYM_OK;
}

int chym_split3_bf16(const float *x, int64_t n, uint16_t *hi, uint16_t *mid, uint16_t *lo, chym_stream_t stream) {
    if (n < 0 || n % 8) return fail(CHYM_EINVAL, "n = %lld must be a non-negative multiple of 8", (long long)n);
    if (!x || !hi || !mid || !lo) return fail(CHYM_EINVAL, "pointers must not be NULL");
    if ((uintptr_t)hi % 16 || (uintptr_t)mid % 16 || (uintptr_t)lo % 16)
        return fail(CHYM_EINVAL, "hi, mid and lo must be 16-byte aligned");
    if (n == 0) return CHYM_OK;
    int rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_split3(x, n, hi, mid, lo, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "split launch");
}

// ----------------------------------------------------------- learned restart
int chym_sign_words(int32_t n, int32_t d, int32_t r, const float *x, uint64_t *words, chym_stream_t stream) {
    int rc = validate_sizes(n, d, r);
    if (rc) return rc;
    if (!x || !words) return fail(CHYM_EINVAL, "x and words must not be NULL");
    rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_sign_words(n, d, r, x, words, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "sign words launch");
}

int chym_features(int32_t n, int32_t d, int32_t r, const void *j, int32_t j_dtype, const float *x,
                  uint64_t *prev_words, float *features, int32_t checkpoint, chym_stream_t stream) {
    int rc = validate_sizes(n, d, r);
    if (rc) return rc;
    if (n > 8192) return fail(CHYM_EUNSUPPORTED, "features need n <= 8192");
    if (j_dtype == CHYM_J_ELL) return fail(CHYM_EUNSUPPORTED, "features take dense couplings");
    if (!valid_jdtype(j_dtype)) return fail(CHYM_EINVAL, "bad j_dtype %d", j_dtype);
    if (!j || !x || !prev_words || !features) return fail(CHYM_EINVAL, "pointers must not be NULL");
    if (checkpoint < 0 || 4 * checkpoint + 4 > CHYM_FEATURES)
        return fail(CHYM_EINVAL, "checkpoint = %d must be in 0..%d", checkpoint, CHYM_FEATURES / 4 - 1);
    rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_features(n, d, r, j, j_dtype, x, prev_words, features, CHYM_FEATURES, 4 * checkpoint,
                                         (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "features launch");
}

int chym_feature_standardize(int32_t groups, int32_t group, const float *in, float *out, chym_stream_t stream) {
    if (groups < 1 || group < 1) return fail(CHYM_EINVAL, "groups = %d and group = %d must be >= 1", groups, group);
    if (!in || !out) return fail(CHYM_EINVAL, "pointers must not be NULL");
    if ((long long)groups * group * CHYM_FEATURES > (1ll << 31))
        return fail(CHYM_EUNSUPPORTED, "at most 2^31 feature values");
    int rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_standardize(groups, group, in, out, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "standardize launch");
}

int chym_select_top(int32_t groups, int32_t group, int32_t keep, const float *score, int32_t *idx,
                    chym_stream_t stream) {
    if (groups < 1 || group < 1) return fail(CHYM_EINVAL, "groups = %d and group = %d must be >= 1", groups, group);
    if (keep < 1 || keep > group) return fail(CHYM_EINVAL, "keep = %d must be in 1..group (%d)", keep, group);
    if (!score || !idx) return fail(CHYM_EINVAL, "pointers must not be NULL");
    if ((long long)groups * group > (1ll << 31) - 1) return fail(CHYM_EUNSUPPORTED, "at most 2^31 - 1 scores");
    int rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_select_top(groups, group, keep, score, idx, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "select launch");
}

int chym_gather_replicas(int32_t n, int32_t d, int32_t r_src, const float *x_src, const float *pump_src, int32_t m,
                         const int32_t *idx, float *x_dst, float *pump_dst, chym_stream_t stream) {
    int rc = validate_sizes(n, d, r_src);
    if (rc) return rc;
    if (m < 0) return fail(CHYM_EINVAL, "m = %d must be >= 0", m);
    if (!x_src || !idx || !x_dst || (pump_dst && !pump_src)) return fail(CHYM_EINVAL, "pointers must not be NULL");
    if (m == 0) return CHYM_OK;
    rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_gather_replicas(n, d, r_src, x_src, pump_src, m, idx, x_dst, pump_dst,
                                                (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "gather launch");
}

int chym_mlp_scratch_floats(int32_t batch, size_t *floats) {
    if (!floats || batch < 0) return fail(CHYM_EINVAL, "bad arguments");
    *floats = chym::mlp_backward_scratch_floats(batch);
    return CHYM_OK;
}

int chym_mlp_forward(int32_t batch, const float *features, const uint16_t *w_bf16, float *logit, float *h1, float *h2,
                     chym_stream_t stream) {
    if (batch < 0) return fail(CHYM_EINVAL, "batch = %d must be >= 0", batch);
    if (!features || !w_bf16 || !logit) return fail(CHYM_EINVAL, "features, weights and logit must not be NULL");
    if ((h1 == nullptr) != (h2 == nullptr)) return fail(CHYM_EINVAL, "h1 and h2 must both be given or both NULL");
    if (batch == 0) return CHYM_OK;
    int rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_mlp_forward(batch, features, w_bf16, logit, h1, h2, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "mlp forward launch");
}

int chym_mlp_backward(int32_t batch, const float *features, const float *labels, const uint16_t *w_bf16,
                      const float *logit, const float *h1, const float *h2, float *scratch, float *grad, float *loss,
                      chym_stream_t stream) {
    if (batch < 1) return fail(CHYM_EINVAL, "batch = %d must be >= 1", batch);
    if (!features || !labels || !w_bf16 || !logit || !h1 || !h2 || !scratch || !grad || !loss)
        return fail(CHYM_EINVAL, "pointers must not be NULL");
    int rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_mlp_backward(batch, features, labels, w_bf16, logit, h1, h2, scratch, grad, loss,
                                             (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "mlp backward launch");
}

int chym_mlp_adam(float *w_master, uint16_t *w_bf16, float *m, float *v, const float *grad, float lr, float beta1,
                  float beta2, float eps, int32_t t, chym_stream_t stream) {
    if (!w_master || !w_bf16 || !m || !v || !grad) return fail(CHYM_EINVAL, "pointers must not be NULL");
    if (t < 1) return fail(CHYM_EINVAL, "t = %d must be >= 1", t);
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(CHYM_EINVAL, "bad Adam hyper-parameters");
    int rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_mlp_adam(w_master, w_bf16, m, v, grad, lr, beta1, beta2, eps, t, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "adam launch");
}

int chym_to_bf16(const float *src, uint16_t *dst, int32_t n, chym_stream_t stream) {
    if (!src || !dst || n < 0) return fail(CHYM_EINVAL, "bad arguments");
    if (n == 0) return CHYM_OK;
    int rc = check_device();
    if (rc) return rc;
    hipError_t e = chym::launch_to_bf16(src, dst, n, (hipStream_t)stream);
    return e == hipSuccess ? CHYM_OK : hip_fail(e, "bf16 launch");
}

int chym_plan_save(const char *path) {
    if (!path) return fail(CHYM_EINVAL, "path is NULL");
    FILE *f = fopen(path, "w");
    if (!f) return fail(CHYM_EINVAL, "cannot open %s for writing", path);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    fprintf(f, "# libchym plan table: tiles d xs js kernel waves ms\n");
    for (const auto &kv : g_plan)
        fprintf(f, "%d %d %d %d %d %d %.4f\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                std::get<3>(kv.first), code_of_kind(kv.second.kind),
                kv.second.waves, kv.second.ms);
    fclose(f);
    return CHYM_OK;
}

int chym_plan_load(const char *path) {
    if (!path) return fail(CHYM_EINVAL, "path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return fail(CHYM_EINVAL, "cannot open %s", path);
    char line[256];
    std::vector<std::pair<VariantKey, PlanValue>> got;
    int lineno = 0;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        if (line[0] == '#' || line[0] == '\n') continue;
        int t, d, xs, js, kernel, waves;
        float ms;
        if (sscanf(line, "%d %d %d %d %d %d %f", &t, &d, &xs, &js, &kernel, &waves, &ms) != 7 || t < 1 || d < 1 ||
            d > 4 || (xs != 1 && xs != 3) || (js != 1 && js != 3) ||
            !valid_kernel_code(kernel) ||
            (kernel == CHYM_KERNEL_SLAB ? (waves != chym::kSlabWaves8 && waves != chym::kSlabWaves16)
                                        : (waves < 1 || waves > 4))) {
            fclose(f);
            return fail(CHYM_EINVAL, "%s:%d: malformed plan entry", path, lineno);
        }
        const VariantKey k = std::make_tuple(t, d, xs, js);
        const bool built = kernel == CHYM_KERNEL_SLAB ? chym::slab_shape_exists(t, d, xs, js, waves)
                                                      : chym::persistent_kind_exists(t, d, xs, js, kind_of_code(kernel));
        if (key_is_slab(k) != (kernel == CHYM_KERNEL_SLAB) || !built) {
            fclose(f);
            return fail(CHYM_EINVAL, "%s:%d: kernel %d does not run %d tiles at d = %d in this form", path, lineno,
                        kernel, t, d);
        }
        got.push_back({k, PlanValue{kind_of_code(kernel), waves, ms}});
    }
    fclose(f);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto &kv : got) g_plan[kv.first] = kv.second;
    return CHYM_OK;
}

}  // extern "C"
