// libusp host runtime: the C-ABI of include/usp.h over the gfx950 kernels.
//
// An instance owns two particle buffers (ping-pong) of ncell regions with
// `cap` slots each, per-component arrays (SoA), a bin table per buffer, the
// per-cell moment arrays and four control words (current buffer, step,
// sample count, sticky error).  usp_step enqueues, per step, the fused cell
// kernel, the P_ne kernel and the control kernel for all listed instances at
// once; the first launch of a call only adds/advects (step 2-3) and the last
// only relaxes, so that between calls the state is "every particle in its own
// cell, in canonical order".
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/usp.h"
#include "usp_common.h"

namespace usp {
template <typename real, int DIM, int NT, int PPT, int PPT2, bool XB>
__global__ void cell_kernel(Batch B);
template <typename real, int DIM>
__global__ void init_kernel(Batch B, const double* init_n, const double* init_u,
                            const double* init_T);
__global__ void fields_kernel(Batch B, int init);
__global__ void ctl_kernel(Batch B, int relaxed);
__global__ void philox_kernel(const uint32_t* ctr, uint32_t k0, uint32_t k1, int n,
                              uint32_t* out);
__global__ void fields_out_kernel(Batch B, int which, double* out, int field_major);
}  // namespace usp

using namespace usp;

namespace {

struct Instance {
    InstDev h;            // host copy of the descriptor
    InstDev* d = nullptr; // device copy (single-instance launches)
    int* dbase = nullptr; // {0, ncell}
    std::vector<void*> allocs;
    size_t bytes = 0;
    bool alive = false;
    bool diag_on = false;
    bool sort_ok = false;  // a step has run with diagnostics on since the last state load
    // diagnostic buffers, kept while diagnostics are switched off and on
    double* dg_mem = nullptr;
    uint32_t* ori_mem[2] = {nullptr, nullptr};
    uint64_t* sorg_mem = nullptr;
    int first = -1;       // first launch shape (-1: the default)
    double mean_ppc = 0;  // particles per cell of the initial state, mean over cells
    double* fview = nullptr;  // usp_moments buffer [18][ncell]
    int top() const { return pick_shape_index(h.max_ppc); }
    // open faces or the plate: the kernel variant with the extended boundary set
    int xb() const { return (h.open_mask != 0 || h.plate) ? 1 : 0; }
    // Default first shape: cells of up to about 170 particles on average
    // (their count grows by a third with the weighted particles, plus the
    // added batches) go to one wave with 4 slots per lane, up to about 250
    // (without open faces or the plate) to one wave with 6; denser instances
    // to the workgroup shapes.
    int default_first() const
    {
        if (mean_ppc * 1.4 + 16.0 <= SHAPES[SHAPE_W4].slots()) return SHAPE_W4;
        if (!xb() && mean_ppc * 1.4 + 24.0 <= SHAPES[SHAPE_W6].slots()) return SHAPE_W6;
        return std::min(top(), TIER_FIRST);
    }
    int first_shape() const { return first >= 0 ? first : default_first(); }
};

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of usp_step_noalloc: one call's batch descriptor table, the
// instance base offsets of each launch group and the shape-tier lists, in a
// device array of the code object (one copy per device, held until the
// process ends).  In host code `scratch` names a host-side stand-in, not the
// device array: its device address is taken once per device with
// hipGetSymbolAddress (usp_create) and only that address reaches kernels.
// ---------------------------------------------------------------------------
namespace {
constexpr int NA_MAX_INST = 1024;       // instances per call
constexpr int NA_MAX_CELLS = 1 << 19;   // cells per call, all instances
constexpr int NA_MAX_DEV = 64;
constexpr size_t na_round(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t NA_TABLE_BYTES = na_round(sizeof(InstDev) * NA_MAX_INST);
// a group of m instances takes m + 1 base entries: at most 2 x NA_MAX_INST
constexpr size_t NA_BASE_BYTES = na_round(sizeof(int) * 2 * NA_MAX_INST);
constexpr size_t NA_TIER_BYTES = na_round(sizeof(int) * NSHAPE * (size_t)(1 + NA_MAX_CELLS));
constexpr size_t NA_BYTES = NA_TABLE_BYTES + NA_BASE_BYTES + NA_TIER_BYTES;
static_assert(sizeof(InstDev) % 4 == 0, "descriptors are copied as 32-bit words");

std::mutex na_mu;
void* na_ptr[NA_MAX_DEV];  // device address of `scratch` per device

// copies instance descriptors into a batch table: block i copies src[i]
constexpr int NA_PACK = 64;
struct DescPack {
    const InstDev* src[NA_PACK];
    int n;
};
}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {
__global__ void na_copy_desc(DescPack pk, InstDev* dst)
{
    const int i = blockIdx.x;
    if (i >= pk.n) return;
    const uint32_t* s = (const uint32_t*)pk.src[i];
    uint32_t* d = (uint32_t*)(dst + i);
    for (int w = threadIdx.x; w < (int)(sizeof(InstDev) / 4); w += blockDim.x) d[w] = s[w];
}

// base offsets of a batch table (base[0] = 0, base[i + 1] = base[i] + ncell
// of instance i) and cleared counts of the group's tier lists
__global__ void na_base_tiers(const InstDev* tbl, int n, int* base, int* tiers, int stride)
{
    if (threadIdx.x == 0) {
        int acc = 0;
        base[0] = 0;
        for (int i = 0; i < n; ++i) {
            acc += tbl[i].ncell;
            base[i + 1] = acc;
        }
    }
    if (threadIdx.x < NSHAPE) tiers[(size_t)threadIdx.x * stride] = 0;
}
}  // namespace

struct usp_ctx {
    usp_device dev;
    hipStream_t stream = nullptr;
    std::vector<Instance*> inst;
    std::string err;
    int block = 256;
    size_t allocated = 0;
    // kernel timing: a start/stop event pair per cell-kernel launch
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    long long timed_passes = 0;
    // device descriptor tables of launch groups, keyed by their instance ids,
    // with the group's shape-tier lists (NSHAPE x (1 + ncells) ints)
    struct Group {
        InstDev* d = nullptr;
        int* base = nullptr;
        size_t bytes = 0;
        int* tiers = nullptr;
        size_t tier_bytes = 0;
    };
    std::map<std::vector<int>, Group> groups;
    // shape-tier lists of single-instance launches (initial / loaded states)
    int* tiers = nullptr;
    int tier_cells = 0;
    // dynamic LDS limit already set per kernel
    std::map<const void*, size_t> lds_set;
    // concurrent launch groups: one side stream each (default priority),
    // forked from and joined back to the caller's stream with events
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    // device address of the static scratch array (usp_step_noalloc)
    void* scratch = nullptr;
    // graph replay of whole usp_step calls, keyed by (instance ids, steps)
    bool graph = false;
    hipStream_t cap = nullptr;
    std::map<std::vector<int>, hipGraphExec_t> graphs;
};

namespace {

usp_status fail(usp_ctx* ctx, usp_status s, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    return s;
}

#define HIPCHK(ctx, call)                                                               \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(ctx, USP_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

void* dalloc(usp_ctx* ctx, size_t bytes)
{
    void* p = nullptr;
    if (bytes == 0) bytes = 16;
    if (ctx->dev.budget && ctx->allocated + bytes > ctx->dev.budget) return nullptr;
    if (ctx->dev.alloc) {
        p = ctx->dev.alloc(bytes, ctx->dev.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) ctx->allocated += bytes;
    return p;
}

void dfree(usp_ctx* ctx, void* p, size_t bytes)
{
    if (!p) return;
    if (ctx->dev.free) ctx->dev.free(p, ctx->dev.user);
    else (void)hipFree(p);
    ctx->allocated -= std::min(ctx->allocated, bytes);
}

struct Window {
    int Kx, Ky;
};

int axis_limit(int n, bool periodic, int hard)
{
    int lim = periodic ? n / 2 : n - 1;
    if (lim < 0) lim = 0;
    return std::min(lim, hard);
}

// Half width of the sort window: the largest displacement in cells that a
// particle of the initial state or a wall emission can make in one step,
// from a six-sigma thermal speed plus the largest drift, with 30 % margin.
Window choose_window(const usp_gas* gas, const usp_problem* pb, const usp_numerics* nm,
                     const double* init_u, const double* init_T)
{
    const int ncell = pb->nx * pb->ny;
    double vmax = 0.0;
    for (int c = 0; c < ncell; ++c) {
        const double* u = init_u + 3 * c;
        const double s = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) +
                         6.0 * sqrt(gas->kB * init_T[c] / gas->m);
        vmax = std::max(vmax, s);
    }
    for (int f = 0; f < 4; ++f) {
        const double* u = pb->face[f].u;
        const double s = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) +
                         6.0 * sqrt(gas->kB * pb->face[f].T / gas->m);
        vmax = std::max(vmax, s);
    }
    vmax *= 1.3;
    Window w;
    const bool px = pb->face[0].kind == USP_BC_PERIODIC, py = pb->face[2].kind == USP_BC_PERIODIC;
    // cells crossed in one step at vmax, held below the axis limit before it
    // becomes an int (a speed far beyond the grid must not wrap the count)
    auto reach_cells = [&](double inv_d, int limit) {
        const double k = ceil(vmax * nm->dt * inv_d) + 1.0;
        return k < (double)limit ? (int)k : limit;
    };
    if (pb->dim == 1) {
        const int lim = axis_limit(pb->ny, py, 127);
        w.Ky = nm->window > 0 ? std::min(nm->window, lim) : reach_cells(pb->inv_dy, lim);
        w.Kx = 0;
    } else {
        const int limx = axis_limit(pb->nx, px, 7), limy = axis_limit(pb->ny, py, 7);
        w.Kx = nm->window > 0 ? std::min(nm->window, limx) : reach_cells(pb->inv_dx, limx);
        w.Ky = nm->window > 0 ? std::min(nm->window, limy) : reach_cells(pb->inv_dy, limy);
    }
    return w;
}

usp_status validate(usp_ctx* ctx, const usp_gas* gas, const usp_problem* pb, const usp_numerics* nm)
{
    if (!gas || !pb || !nm) return fail(ctx, USP_EINVAL, "null argument");
    if (pb->dim != 1 && pb->dim != 2) return fail(ctx, USP_EINVAL, "dim must be 1 or 2");
    if (pb->nx < 1 || pb->ny < 1 || (pb->dim == 1 && pb->nx != 1))
        return fail(ctx, USP_EINVAL, "bad grid");
    if (!(nm->dt > 0) || !(nm->Np > 0) || !(pb->vcell > 0) || !(nm->r_p > 0))
        return fail(ctx, USP_EINVAL, "dt, Np, vcell and r_p must be positive");
    if (nm->precision != 32 && nm->precision != 64)
        return fail(ctx, USP_EINVAL, "precision must be 32 or 64");
    if (nm->max_ppc < 2 || nm->max_ppc > MAX_PPC)
        return fail(ctx, USP_EINVAL, "max_ppc must be in [2, 2048]");
    if (nm->n_avg < 1) return fail(ctx, USP_EINVAL, "n_avg must be >= 1");
    if ((long long)pb->nx * pb->ny > (1LL << 26)) return fail(ctx, USP_EINVAL, "too many cells");
    // the gather addresses a particle slot of the instance by 31 bits (the
    // top bit marks the far-mover list)
    if ((long long)pb->nx * pb->ny * ((nm->max_ppc + 63) / 64 * 64) >= (1LL << 31))
        return fail(ctx, USP_EINVAL, "cells x capacity must stay below 2^31 particle slots");
    bool open = false;
    for (int f = 0; f < 4; ++f) {
        const usp_face& fc = pb->face[f];
        if (fc.kind < USP_BC_DIFFUSE || fc.kind > USP_BC_OPEN)
            return fail(ctx, USP_EINVAL, "unknown face kind");
        if (fc.kind != USP_BC_OPEN) continue;
        open = true;
        if (!(fc.n >= 0.0) || !(fc.n_b >= 0.0) || !(fc.T > 0.0) || !(fc.T_b > 0.0))
            return fail(ctx, USP_EINVAL, "open face needs n, n_b >= 0 and T, T_b > 0");
        if (fc.u[f / 2] != 0.0)
            return fail(ctx, USP_EINVAL, "open face reservoir moves across the face");
        // expected entering particles per cell and step, n sqrt(kT / (2 pi m))
        // area dt / Np, for both reservoir states: beyond max_ppc every
        // boundary cell would overflow at once (and a count beyond an int
        // would wrap)
        if (pb->dim == 1 && f < 2) continue;
        const double area = pb->dim == 2 ? (f < 2 ? pb->dy : pb->dx) : 1.0;
        for (int b = 0; b < 2; ++b) {
            // the second state only on a split face of a 2-D problem
            if (b == 1 && !(pb->dim == 2 && fc.split < HUGE_VAL)) continue;
            const double n = b ? fc.n_b : fc.n, T = b ? fc.T_b : fc.T;
            const double v = n * sqrt(gas->kB * T / (gas->m * 2.0 * M_PI)) * area * nm->dt / nm->Np;
            if (!(v <= (double)nm->max_ppc))
                return fail(ctx, USP_EINVAL,
                            "an open face would bring more than max_ppc particles into a cell "
                            "per step");
        }
    }
    if ((pb->face[0].kind == USP_BC_PERIODIC) != (pb->face[1].kind == USP_BC_PERIODIC) ||
        (pb->face[2].kind == USP_BC_PERIODIC) != (pb->face[3].kind == USP_BC_PERIODIC))
        return fail(ctx, USP_EINVAL, "a periodic face needs a periodic opposite face");
    // the open-face / plate kernel variant runs in the shapes up to 256 x
    // (4 | 6) slots: its 8-slot shape is switched off (a run of it faulted
    // on the device with the cause not found)
    if ((open || pb->plate) && pick_shape_index(nm->max_ppc) == NSHAPE_WG - 1)
        return fail(ctx, USP_EINVAL,
                    "open faces or the plate: max_ppc must be at most 1365 (8-slot shape off)");
    if (open && (pb->accel[0] != 0.0 || pb->accel[1] != 0.0 || pb->accel[2] != 0.0))
        return fail(ctx, USP_EINVAL, "open faces cannot be combined with a body acceleration");
    // every mode switch takes one of its listed values (no silent default branch)
    if (nm->pne_mode < USP_PNE_FIXED || nm->pne_mode > USP_PNE_GLL_AVG)
        return fail(ctx, USP_EINVAL, "unknown pne_mode");
    if (nm->weight_mode != USP_WEIGHT_CONSISTENT && nm->weight_mode != USP_WEIGHT_LITERAL)
        return fail(ctx, USP_EINVAL, "unknown weight_mode");
    if (nm->conserve_mode != USP_CONSERVE_FULL && nm->conserve_mode != USP_CONSERVE_NONE)
        return fail(ctx, USP_EINVAL, "unknown conserve_mode");
    if (nm->jmom_mode != USP_JMOM_INST && nm->jmom_mode != USP_JMOM_AVG)
        return fail(ctx, USP_EINVAL, "unknown jmom_mode");
    if (nm->spawn_projection != 0 && nm->spawn_projection != 1)
        return fail(ctx, USP_EINVAL, "spawn_projection must be 0 or 1");
    if (nm->avg_init != 0 && nm->avg_init != 1)
        return fail(ctx, USP_EINVAL, "avg_init must be 0 or 1");
    if (nm->window < 0) return fail(ctx, USP_EINVAL, "window must be >= 0");
    if (!(nm->Kn_c > 0.0)) return fail(ctx, USP_EINVAL, "Kn_c must be positive");
    if (nm->scheme != USP_SCHEME_USP && nm->scheme != USP_SCHEME_SP)
        return fail(ctx, USP_EINVAL, "unknown scheme");
    if (nm->es_mode != USP_ES_SAMPLED && nm->es_mode != USP_ES_MEAN)
        return fail(ctx, USP_EINVAL, "unknown es_mode");
    if (nm->gll_u != USP_GLL_U_SOUND && nm->gll_u != USP_GLL_U_LITERAL)
        return fail(ctx, USP_EINVAL, "unknown gll_u");
    if (nm->select_mode != USP_SELECT_BERNOULLI && nm->select_mode != USP_SELECT_COUNT)
        return fail(ctx, USP_EINVAL, "unknown select_mode");
    if (nm->es_sampler != USP_ES_SAMPLER_CHOLESKY && nm->es_sampler != USP_ES_SAMPLER_LINEAR)
        return fail(ctx, USP_EINVAL, "unknown es_sampler");
    if (nm->es_mode == USP_ES_MEAN && !(gas->Pr > 0.0 && gas->Pr != 1.0))
        return fail(ctx, USP_EINVAL, "es_mode MEAN needs 0 < Pr != 1");
    if (nm->scheme == USP_SCHEME_SP && !(nm->pne_mode == USP_PNE_FIXED && nm->pne_fixed == 0.0))
        return fail(ctx, USP_EINVAL, "SP-ESBGK needs pne_mode FIXED with pne_fixed 0");
    if (pb->plate) {
        if (pb->dim != 2 || !(pb->plate_x > pb->x0 && pb->plate_x < pb->x1))
            return fail(ctx, USP_EINVAL, "plate needs 2-D and x0 < plate_x < x1");
        if (!(pb->plate_ylo <= pb->plate_yhi) || !(pb->plate_T > 0.0))
            return fail(ctx, USP_EINVAL, "plate needs plate_ylo <= plate_yhi and plate_T > 0");
    }
    return USP_OK;
}

size_t footprint_of(const usp_problem* pb, const usp_numerics* nm, int nb)
{
    const size_t ncell = (size_t)pb->nx * pb->ny;
    const size_t rb = nm->precision == 32 ? 4 : 8;
    const size_t cap = (size_t)((nm->max_ppc + 63) / 64 * 64);
    size_t b = 0;
    b += 2 * (size_t)(pb->dim + 4) * ncell * cap * rb;  // particles
    b += 2 * ncell * (size_t)(nb + 1) * 4;              // bin tables
    b += 4 * NMOM * ncell * 8;                          // moments
    b += 2 * ncell * 8 + ncell * 4 + 64;                // P_ne, counts, ctl
    const size_t far_cap = std::max((size_t)4096, ncell * 8);
    b += 2 * far_cap * (12 + (size_t)(pb->dim + 4) * rb);  // far-mover lists
    return b;
}

Instance* get_inst(usp_ctx* ctx, int id)
{
    if (!ctx || id < 0 || id >= (int)ctx->inst.size()) return nullptr;
    Instance* in = ctx->inst[id];
    return (in && in->alive) ? in : nullptr;
}

template <typename F>
usp_status with_kernel(int prec, int dim, F f)
{
    if (prec == 32 && dim == 1) return f((float*)nullptr, std::integral_constant<int, 1>());
    if (prec == 32 && dim == 2) return f((float*)nullptr, std::integral_constant<int, 2>());
    if (prec == 64 && dim == 1) return f((double*)nullptr, std::integral_constant<int, 1>());
    return f((double*)nullptr, std::integral_constant<int, 2>());
}

// the shapes with a built kernel; anything else has none (a launch of
// another kernel with this shape's block and LDS sizes would run it outside
// what it assumes)
constexpr bool shape_is_built(Shape sh)
{
    if (sh.nt == 64) return sh.ppt2 == 0 && (sh.ppt == 4 || sh.ppt == 6);
    if (sh.nt != 256) return false;
    if (sh.ppt2 == 6) return sh.ppt == 4;
    return sh.ppt2 == 0 && (sh.ppt == 1 || sh.ppt == 2 || sh.ppt == 4 || sh.ppt == 8);
}

constexpr bool all_shapes_built()
{
    for (int i = 0; i < NSHAPE; ++i)
        if (!shape_is_built(SHAPES[i])) return false;
    return true;
}
static_assert(all_shapes_built(), "every launch shape of the table needs its kernel");

template <typename real, int D, bool XB>
const void* cell_kernel_for(Shape sh)
{
    if (!shape_is_built(sh)) return nullptr;
    if (sh.nt == 64) {
        if (sh.ppt == 4) return (const void*)cell_kernel<real, D, 64, 4, 0, XB>;
        if constexpr (!XB) return (const void*)cell_kernel<real, D, 64, 6, 0, false>;
        return nullptr;  // no 6-slot wave shape with open faces or the plate
    }
    if (sh.ppt2 == 6) return (const void*)cell_kernel<real, D, 256, 4, 6, XB>;
    switch (sh.ppt) {
        case 1: return (const void*)cell_kernel<real, D, 256, 1, 0, XB>;
        case 2: return (const void*)cell_kernel<real, D, 256, 2, 0, XB>;
        case 4: return (const void*)cell_kernel<real, D, 256, 4, 0, XB>;
        case 8: return (const void*)cell_kernel<real, D, 256, 8, 0, XB>;
        default: return nullptr;
    }
}

usp_status ensure_tiers(usp_ctx* ctx, int ncells)
{
    if (ncells <= ctx->tier_cells) return USP_OK;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->tiers) dfree(ctx, ctx->tiers, sizeof(int) * NSHAPE * (size_t)(1 + ctx->tier_cells));
    const size_t bytes = sizeof(int) * NSHAPE * (size_t)(1 + ncells);
    ctx->tiers = (int*)dalloc(ctx, bytes);
    ctx->tier_cells = 0;
    if (!ctx->tiers) return fail(ctx, USP_ENOMEM, "shape tier lists");
    HIPCHK(ctx, hipMemsetAsync(ctx->tiers, 0, bytes, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->tier_cells = ncells;
    return USP_OK;
}

void attach_tiers(usp_ctx* ctx, Batch& B)
{
    B.tiers = ctx->tiers;
    B.tier_stride = 1 + ctx->tier_cells;
}

usp_status set_lds(usp_ctx* ctx, const void* kern, size_t lds)
{
    auto it = ctx->lds_set.find(kern);
    if (it != ctx->lds_set.end() && it->second >= lds) return USP_OK;
    HIPCHK(ctx, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    ctx->lds_set[kern] = lds;
    return USP_OK;
}

// the kernels of one cell pass (the shape chain from `first`) with their
// dynamic LDS sizes: f(position in the chain, chain, its length, shape,
// kernel, lds bytes)
template <typename F>
usp_status for_each_tier(int prec, int dim, int xb, int max_nb, int first, int top, F f)
{
    int chain[NSHAPE];
    const int n = shape_chain(first, top, chain);
    for (int i = 0; i < n; ++i) {
        const Shape sh = SHAPES[chain[i]];
        const size_t lds = lds_bytes(sh.nt, sh.slots(), max_nb);
        usp_status st = with_kernel(prec, dim, [&](auto* rp, auto dimc) -> usp_status {
            using real = std::remove_pointer_t<decltype(rp)>;
            constexpr int D = decltype(dimc)::value;
            return f(i, chain, n, sh,
                     xb ? cell_kernel_for<real, D, true>(sh) : cell_kernel_for<real, D, false>(sh),
                     lds);
        });
        if (st) return st;
    }
    return USP_OK;
}

usp_status prepare_cell(usp_ctx* ctx, int prec, int dim, int xb, int max_nb, int first, int top)
{
    return for_each_tier(prec, dim, xb, max_nb, first, top,
                         [&](int, const int*, int, Shape, const void* kern, size_t lds) {
                             if (!kern)
                                 return fail(ctx, USP_EINVAL,
                                             "launch shape not built for this instance");
                             return set_lds(ctx, kern, lds);
                         });
}

// one cell-kernel pass over the batch (B.tiers set by the caller): the first
// shape of the chain runs every cell; a cell that needs more slots is handed
// on, untouched, to the next shape of the chain through the tier list of
// the shape that handed it on.
usp_status launch_cell(usp_ctx* ctx, Batch B, int prec, int dim, int xb, int max_nb, int first,
                       int top, hipStream_t stream)
{
    // timing: the stream is drained first, so that the pass's launches are
    // queued behind its start event at once and nothing but the pass lies
    // between the two events
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
        HIPCHK(ctx, hipStreamSynchronize(stream));
        HIPCHK(ctx, hipEventCreate(&e0));
        HIPCHK(ctx, hipEventCreate(&e1));
        HIPCHK(ctx, hipEventRecord(e0, stream));
    }
    usp_status st = for_each_tier(
        prec, dim, xb, max_nb, first, top,
        [&](int i, const int* chain, int n, Shape sh, const void* kern,
            size_t lds) -> usp_status {
            if (!kern) return fail(ctx, USP_EINVAL, "launch shape not built for this instance");
            usp_status s2 = set_lds(ctx, kern, lds);
            if (s2) return s2;
            B.tier_in = i == 0 ? nullptr : B.tiers + (size_t)chain[i - 1] * B.tier_stride;
            B.tier_out = i + 1 == n ? nullptr : B.tiers + (size_t)chain[i] * B.tier_stride;
            void* args[] = {(void*)&B};
            HIPCHK(ctx, hipLaunchKernel(kern, dim3(B.ncells), dim3(sh.nt), args, lds, stream));
            return USP_OK;
        });
    if (st) return st;
    if (ctx->timing) {
        HIPCHK(ctx, hipEventRecord(e1, stream));
        ctx->events.emplace_back(e0, e1);
    }
    if (ctx->timing) ++ctx->timed_passes;
    return USP_OK;
}

usp_status launch_fields(usp_ctx* ctx, const Batch& B, int init, hipStream_t stream)
{
    const int nt = 256;
    hipLaunchKernelGGL(fields_kernel, dim3((B.ncells + nt - 1) / nt), dim3(nt), 0, stream, B,
                       init);
    HIPCHK(ctx, hipGetLastError());
    return USP_OK;
}

usp_status launch_ctl(usp_ctx* ctx, const Batch& B, int relaxed, hipStream_t stream)
{
    hipLaunchKernelGGL(ctl_kernel, dim3((B.ninst + 63) / 64), dim3(64), 0, stream, B, relaxed);
    HIPCHK(ctx, hipGetLastError());
    return USP_OK;
}

Batch single_batch(Instance* in, int mode)
{
    Batch B;
    B.inst = in->d;
    B.base = in->dbase;
    B.ninst = 1;
    B.ncells = in->h.ncell;
    B.mode = mode;
    return B;
}

usp_status upload_desc(usp_ctx* ctx, Instance* in)
{
    HIPCHK(ctx, hipMemcpyAsync(in->d, &in->h, sizeof(InstDev), hipMemcpyHostToDevice, ctx->stream));
    return USP_OK;
}

usp_status read_ctl(usp_ctx* ctx, Instance* in, int* ctl)
{
    HIPCHK(ctx, hipMemcpyAsync(ctl, in->h.ctl, sizeof(int) * CTL_N, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return USP_OK;
}

usp_status err_status(usp_ctx* ctx, int e)
{
    if (e & ERR_CAPACITY) return fail(ctx, USP_ECAPACITY, "a cell exceeded max_ppc particles");
    if (e & ERR_WINDOW)
        return fail(ctx, USP_EWINDOW, "a particle moved farther than the sort window");
    if (e & ERR_NONFINITE)
        return fail(ctx, USP_ENONFINITE, "a cell moment became infinite or not a number");
    return USP_OK;
}

void drop_groups(usp_ctx* ctx)
{
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
    for (auto& kv : ctx->groups) {
        dfree(ctx, kv.second.d, kv.second.bytes);
        dfree(ctx, kv.second.base, 0);
        dfree(ctx, kv.second.tiers, kv.second.tier_bytes);
    }
    ctx->groups.clear();
}

// moments of the current state + P_ne from them (initial / loaded states)
usp_status finish_state(usp_ctx* ctx, Instance* in)
{
    Batch B = single_batch(in, MODE_MOMENTS);
    usp_status s = ensure_tiers(ctx, B.ncells);
    if (s) return s;
    attach_tiers(ctx, B);
    if ((s = launch_cell(ctx, B, in->h.prec, in->h.dim, in->xb(), in->h.nb, in->first_shape(),
                         in->top(), ctx->stream)))
        return s;
    if ((s = launch_fields(ctx, B, 1, ctx->stream))) return s;
    return launch_ctl(ctx, B, 0, ctx->stream);
}

}  // namespace

extern "C" {

usp_status usp_create(const usp_device* dev, usp_ctx** out)
{
    if (!out) return USP_EINVAL;
    usp_ctx* ctx = new usp_ctx();
    if (dev) ctx->dev = *dev;
    else memset(&ctx->dev, 0, sizeof(ctx->dev));
    ctx->stream = (hipStream_t)ctx->dev.stream;
    if (hipSetDevice(ctx->dev.device) != hipSuccess) {
        delete ctx;
        return USP_EDEVICE;
    }
    if (ctx->dev.device < 0 || ctx->dev.device >= NA_MAX_DEV) {
        delete ctx;
        return USP_EINVAL;
    }
    {
        // the scratch array's address on this device (the device is current)
        std::lock_guard<std::mutex> lock(na_mu);
        void*& p = na_ptr[ctx->dev.device];
        if (!p) {
            void* q = nullptr;
            if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) {
                delete ctx;
                return USP_EDEVICE;
            }
            p = q;
        }
        ctx->scratch = p;
    }
    *out = ctx;
    return USP_OK;
}

void usp_destroy(usp_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (size_t i = 0; i < ctx->inst.size(); ++i)
        if (ctx->inst[i] && ctx->inst[i]->alive) usp_instance_free(ctx, (int)i);
    for (Instance* in : ctx->inst) delete in;
    drop_groups(ctx);
    if (ctx->tiers) dfree(ctx, ctx->tiers, sizeof(int) * NSHAPE * (size_t)(1 + ctx->tier_cells));
    for (size_t i = 0; i < ctx->side.size(); ++i) {
        (void)hipStreamDestroy(ctx->side[i]);
        (void)hipEventDestroy(ctx->join[i]);
    }
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    delete ctx;
}

const char* usp_last_error(usp_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

usp_status usp_footprint(const usp_problem* pb, const usp_numerics* nm, size_t* bytes_out)
{
    if (!pb || !nm || !bytes_out) return USP_EINVAL;
    const int nb = pb->dim == 1 ? 255 : 225;
    *bytes_out = footprint_of(pb, nm, nb);
    return USP_OK;
}

usp_status usp_instance_init(usp_ctx* ctx, const usp_gas* gas, const usp_problem* pb,
                             const usp_numerics* nm, const double* init_n, const double* init_u,
                             const double* init_T, int* id_out)
{
    if (!ctx) return USP_EINVAL;
    usp_status s = validate(ctx, gas, pb, nm);
    if (s) return s;
    if (!init_n || !init_u || !init_T || !id_out) return fail(ctx, USP_EINVAL, "null init field");
    // the initial state: a finite, non-negative particle count (n V / Np, the
    // device rounds it), temperature and velocity in every cell
    for (long long c = 0; c < (long long)pb->nx * pb->ny; ++c) {
        const double v = init_n[c] * pb->vcell / nm->Np;
        if (!(v >= 0.0 && v < 1.0e9))
            return fail(ctx, USP_EINVAL, "init_n must give a finite, non-negative count per cell");
        if (!(init_T[c] >= 0.0 && init_T[c] < HUGE_VAL))
            return fail(ctx, USP_EINVAL, "init_T must be finite and non-negative");
        for (int k = 0; k < 3; ++k)
            if (!(fabs(init_u[3 * c + k]) < HUGE_VAL))
                return fail(ctx, USP_EINVAL, "init_u must be finite");
    }
    HIPCHK(ctx, hipSetDevice(ctx->dev.device));
    Instance* in = new Instance();
    InstDev& h = in->h;
    memset(&h, 0, sizeof(h));
    h.m = gas->m;
    h.kB = gas->kB;
    h.mu_ref = gas->mu_ref;
    h.T_ref = gas->T_ref;
    h.omega = gas->omega;
    h.Pr = gas->Pr;
    h.R = gas->kB / gas->m;
    h.F = gas->m * nm->Np / pb->vcell;
    h.dim = pb->dim;
    h.nx = pb->nx;
    h.ny = pb->ny;
    h.ncell = pb->nx * pb->ny;
    h.x0 = pb->x0;
    h.x1 = pb->x1;
    h.y0 = pb->y0;
    h.y1 = pb->y1;
    h.dx = pb->dx;
    h.dy = pb->dy;
    h.inv_dx = pb->inv_dx;
    h.inv_dy = pb->inv_dy;
    h.vcell = pb->vcell;
    h.Np = nm->Np;
    for (int f = 0; f < 4; ++f) {
        h.face_kind[f] = pb->face[f].kind;
        h.face_T[f] = pb->face[f].T;
        for (int k = 0; k < 3; ++k) h.face_u[3 * f + k] = pb->face[f].u[k];
        h.face_n[f] = pb->face[f].n;
        h.face_split[f] = pb->face[f].split;
        h.face_nb[f] = pb->face[f].n_b;
        h.face_Tb[f] = pb->face[f].T_b;
        // x faces of a 1-D problem are inert
        if (pb->face[f].kind == USP_BC_OPEN && (pb->dim == 2 || f >= 2)) h.open_mask |= 1 << f;
    }
    for (int k = 0; k < 3; ++k) h.accel[k] = pb->accel[k];
    h.plate = pb->plate != 0;
    h.plate_x = pb->plate_x;
    h.plate_ylo = pb->plate_ylo;
    h.plate_yhi = pb->plate_yhi;
    h.plate_T = pb->plate_T;
    h.dt = nm->dt;
    h.r_p = nm->r_p;
    h.Kn_c = nm->Kn_c;
    h.pne_fixed = nm->pne_fixed;
    h.pne_mode = nm->pne_mode;
    h.n_avg = nm->n_avg;
    h.avg_start = nm->avg_start;
    h.prec = nm->precision;
    h.weight_mode = nm->weight_mode;
    h.conserve_mode = nm->conserve_mode;
    h.max_ppc = nm->max_ppc;
    h.jmom_mode = nm->jmom_mode;
    h.proj = nm->spawn_projection;
    h.avg_init = nm->avg_init != 0;
    h.scheme = nm->scheme;
    h.es_mode = nm->es_mode;
    h.gll_u = nm->gll_u;
    h.select_mode = nm->select_mode;
    h.es_sampler = nm->es_sampler;
    h.key0 = (uint32_t)(nm->seed & 0xFFFFFFFFu);
    h.key1 = (uint32_t)(nm->seed >> 32);
    Window w = choose_window(gas, pb, nm, init_u, init_T);
    h.Kx = w.Kx;
    h.Ky = w.Ky;
    h.nbx = 2 * w.Kx + 1;
    h.nb = (2 * w.Ky + 1) * h.nbx;
    if (h.nb > MAX_BINS) return fail(ctx, USP_EINVAL, "sort window larger than 256 bins");
    h.cap = (nm->max_ppc + 63) / 64 * 64;
    {
        double tot = 0.0;
        for (int c = 0; c < h.ncell; ++c) tot += floor(init_n[c] * pb->vcell / nm->Np + 0.5);
        in->mean_ppc = tot / h.ncell;
    }

    const size_t ncell = (size_t)h.ncell;
    const size_t rb = h.prec == 32 ? 4 : 8;
    auto A = [&](size_t bytes) -> void* {
        void* p = dalloc(ctx, bytes);
        if (p) {
            in->allocs.push_back(p);
            in->bytes += bytes;
        }
        return p;
    };
    bool ok = true;
    for (int b = 0; b < 2; ++b) {
        for (int k = 0; k < 6; ++k) {
            if (k == 0 && h.dim == 1) {
                h.pc[b][k] = nullptr;
                continue;
            }
            h.pc[b][k] = A(ncell * h.cap * rb);
            ok = ok && h.pc[b][k];
        }
        h.tab[b] = (uint32_t*)A(ncell * (h.nb + 1) * 4);
        ok = ok && h.tab[b];
    }
    h.far_cap = (int)std::max((size_t)4096, ncell * 8);
    h.far_n = (int*)A(2 * sizeof(int));
    ok = ok && h.far_n;
    for (int b = 0; b < 2; ++b) {
        h.far_meta[b] = (uint32_t*)A((size_t)h.far_cap * 12);
        ok = ok && h.far_meta[b];
        for (int k = 0; k < 6; ++k) {
            if (k == 0 && h.dim == 1) {
                h.far_pc[b][k] = nullptr;
                continue;
            }
            h.far_pc[b][k] = A((size_t)h.far_cap * rb);
            ok = ok && h.far_pc[b][k];
        }
    }
    h.mom = (double*)A(NMOM * ncell * 8);
    h.raw = (double*)A(NMOM * ncell * 8);
    h.avg = (double*)A(NMOM * ncell * 8);
    h.avgs = (double*)A(NMOM * ncell * 8);
    h.pcur = (double*)A(ncell * 8);
    h.pprev = (double*)A(ncell * 8);
    h.cnt = (int*)A(ncell * 4);
    h.ctl = (int*)A(CTL_N * 4);
    in->d = (InstDev*)A(sizeof(InstDev));
    in->dbase = (int*)A(2 * sizeof(int));
    ok = ok && h.mom && h.raw && h.avg && h.avgs && h.pcur && h.pprev && h.cnt && h.ctl && in->d &&
         in->dbase;
    if (!ok) {
        for (void* p : in->allocs) dfree(ctx, p, 0);
        ctx->allocated -= std::min(ctx->allocated, in->bytes);
        delete in;
        return fail(ctx, USP_ENOMEM, "device allocation failed or over budget");
    }
    if (h.avg_init) {
        // raw sums of the initial Maxwellian of each cell (N particles at
        // u, theta): N, N u, N (u u + theta I), N (|u|^2 + 5 theta) u
        std::vector<double> A0((size_t)NMOM * ncell);
        for (size_t c = 0; c < ncell; ++c) {
            const double N = (double)(int)floor(init_n[c] * pb->vcell / nm->Np + 0.5);
            const double sq = sqrt(gas->kB * init_T[c] / gas->m), th = sq * sq;
            const double* u = init_u + 3 * c;
            const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            double a[NMOM];
            a[0] = N;
            for (int k = 0; k < 3; ++k) a[1 + k] = N * u[k];
            a[4] = N * (u[0] * u[0] + th);
            a[5] = N * (u[1] * u[1] + th);
            a[6] = N * (u[2] * u[2] + th);
            a[7] = N * u[0] * u[1];
            a[8] = N * u[0] * u[2];
            a[9] = N * u[1] * u[2];
            for (int k = 0; k < 3; ++k) a[10 + k] = N * (u2 + 5.0 * th) * u[k];
            for (int q = 0; q < NMOM; ++q) A0[(size_t)q * ncell + c] = a[q];
        }
        HIPCHK(ctx, hipMemcpyAsync(h.avg, A0.data(), NMOM * ncell * 8, hipMemcpyHostToDevice,
                                   ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(h.avgs, A0.data(), NMOM * ncell * 8, hipMemcpyHostToDevice,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    } else {
        HIPCHK(ctx, hipMemsetAsync(h.avg, 0, NMOM * ncell * 8, ctx->stream));
        HIPCHK(ctx, hipMemsetAsync(h.avgs, 0, NMOM * ncell * 8, ctx->stream));
    }
    HIPCHK(ctx, hipMemsetAsync(h.ctl, 0, CTL_N * 4, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(h.far_n, 0, 2 * sizeof(int), ctx->stream));
    // per-cell records start defined: nothing of a previous user of this
    // memory can reach a kernel
    HIPCHK(ctx, hipMemsetAsync(h.mom, 0, NMOM * ncell * 8, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(h.raw, 0, NMOM * ncell * 8, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(h.pcur, 0, ncell * 8, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(h.pprev, 0, ncell * 8, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(h.cnt, 0, ncell * 4, ctx->stream));
    int base[2] = {0, h.ncell};
    HIPCHK(ctx, hipMemcpyAsync(in->dbase, base, sizeof(base), hipMemcpyHostToDevice, ctx->stream));
    if ((s = upload_desc(ctx, in))) return s;

    // Table 2 step 1
    double *dn = nullptr, *du = nullptr, *dT = nullptr;
    HIPCHK(ctx, hipMalloc(&dn, ncell * 8));
    HIPCHK(ctx, hipMalloc(&du, 3 * ncell * 8));
    HIPCHK(ctx, hipMalloc(&dT, ncell * 8));
    HIPCHK(ctx, hipMemcpyAsync(dn, init_n, ncell * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(du, init_u, 3 * ncell * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(dT, init_T, ncell * 8, hipMemcpyHostToDevice, ctx->stream));
    Batch B = single_batch(in, MODE_MOMENTS);
    s = with_kernel(h.prec, h.dim, [&](auto* rp, auto dimc) -> usp_status {
        using real = std::remove_pointer_t<decltype(rp)>;
        constexpr int D = decltype(dimc)::value;
        hipLaunchKernelGGL((init_kernel<real, D>), dim3(h.ncell), dim3(256), 0, ctx->stream, B, dn,
                           du, dT);
        HIPCHK(ctx, hipGetLastError());
        return USP_OK;
    });
    if (s) return s;
    if ((s = finish_state(ctx, in))) return s;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(dn);
    (void)hipFree(du);
    (void)hipFree(dT);
    in->alive = true;
    ctx->inst.push_back(in);
    *id_out = (int)ctx->inst.size() - 1;
    drop_groups(ctx);
    int ctl[CTL_N];
    if ((s = read_ctl(ctx, in, ctl))) return s;
    return err_status(ctx, ctl[CTL_ERR]);
}

usp_status usp_instance_free(usp_ctx* ctx, int id)
{
    Instance* in = get_inst(ctx, id);
    if (!in) return fail(ctx, USP_ESTATE, "unknown instance");
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : in->allocs) dfree(ctx, p, 0);
    ctx->allocated -= std::min(ctx->allocated, in->bytes);
    in->allocs.clear();
    in->fview = nullptr;
    in->dg_mem = nullptr;
    in->ori_mem[0] = in->ori_mem[1] = nullptr;
    in->sorg_mem = nullptr;
    in->alive = false;
    drop_groups(ctx);
    return USP_OK;
}

usp_status usp_set_block(usp_ctx* ctx, int threads)
{
    if (!ctx) return USP_EINVAL;
    if (threads == 0) threads = 256;
    if (threads != 256) return fail(ctx, USP_EINVAL, "the cell kernel runs 256 threads per cell");
    ctx->block = threads;
    return USP_OK;
}

}  // extern "C"

namespace {

// one launch group of a usp_step call: instances of one kernel flavour
struct Plan {
    Batch B;
    int prec, dim, xb, max_nb, first, top;
};

// groups the instances by kernel flavour (precision, dimension, shape) and
// makes sure their descriptor tables, tier lists and kernel attributes exist
// (all of it before any launch: a graph capture may follow)
usp_status make_plan(usp_ctx* ctx, const int* ids, int n_ids, std::vector<Plan>& plans)
{
    std::vector<char> seen(ctx->inst.size(), 0);
    for (int i = 0; i < n_ids; ++i) {
        if (!get_inst(ctx, ids[i])) return fail(ctx, USP_ESTATE, "unknown or freed instance in step");
        if (seen[ids[i]]++) return fail(ctx, USP_EINVAL, "an instance listed twice in one step");
    }
    // flavour = (precision, dimension, boundary set, first shape, last
    // shape); the map keeps the groups in a fixed order
    std::map<std::vector<int>, std::vector<int>> flavours;
    for (int i = 0; i < n_ids; ++i) {
        Instance* in = get_inst(ctx, ids[i]);
        flavours[{in->h.prec, in->h.dim, in->xb(), in->first_shape(), in->top()}].push_back(
            ids[i]);
    }
    for (auto& fv : flavours) {
        const int prec = fv.first[0], dim = fv.first[1], xb = fv.first[2];
        const int first = fv.first[3], top = fv.first[4];
        const std::vector<int>& sel = fv.second;
        int ncells = 0, max_nb = 0;
        for (int id : sel) {
            ncells += ctx->inst[id]->h.ncell;
            max_nb = std::max(max_nb, ctx->inst[id]->h.nb);
        }
        std::vector<int> key = sel;
        key.push_back(-1 - (first * NSHAPE + top) * 4 - (prec == 64 ? 2 : 0) - (dim - 1));
        auto it = ctx->groups.find(key);
        if (it == ctx->groups.end()) {
            usp_ctx::Group G;
            G.bytes = sizeof(InstDev) * sel.size();
            G.d = (InstDev*)dalloc(ctx, G.bytes);
            G.base = (int*)dalloc(ctx, sizeof(int) * (sel.size() + 1));
            G.tier_bytes = sizeof(int) * NSHAPE * (size_t)(1 + ncells);
            G.tiers = (int*)dalloc(ctx, G.tier_bytes);
            if (!G.d || !G.base || !G.tiers) {
                dfree(ctx, G.d, G.bytes);
                dfree(ctx, G.base, 0);
                dfree(ctx, G.tiers, G.tier_bytes);
                return fail(ctx, USP_ENOMEM, "batch table");
            }
            std::vector<InstDev> hd;
            std::vector<int> base(1, 0);
            for (int id : sel) {
                hd.push_back(ctx->inst[id]->h);
                base.push_back(base.back() + ctx->inst[id]->h.ncell);
            }
            HIPCHK(ctx, hipMemcpyAsync(G.d, hd.data(), G.bytes, hipMemcpyHostToDevice,
                                       ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(G.base, base.data(), sizeof(int) * base.size(),
                                       hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(ctx, hipMemsetAsync(G.tiers, 0, G.tier_bytes, ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            it = ctx->groups.emplace(key, G).first;
        }
        Plan P;
        P.B.inst = it->second.d;
        P.B.base = it->second.base;
        P.B.ninst = (int)sel.size();
        P.B.ncells = ncells;
        P.B.tiers = it->second.tiers;
        P.B.tier_stride = 1 + ncells;
        P.prec = prec;
        P.dim = dim;
        P.xb = xb;
        P.max_nb = max_nb;
        P.first = first;
        P.top = top;
        usp_status st = prepare_cell(ctx, prec, dim, xb, max_nb, first, top);
        if (st) return st;
        plans.push_back(P);
    }
    return USP_OK;
}

// the launches of nsteps steps of one group on one stream: a move pass, then
// per step a relax (+ move) pass, the P_ne field and the step control
usp_status enqueue_group(usp_ctx* ctx, Plan P, int nsteps, hipStream_t st)
{
    usp_status s;
    P.B.mode = MODE_MOVE;
    if ((s = launch_cell(ctx, P.B, P.prec, P.dim, P.xb, P.max_nb, P.first, P.top, st))) return s;
    if ((s = launch_ctl(ctx, P.B, 0, st))) return s;
    for (int k = 0; k < nsteps; ++k) {
        P.B.mode = k + 1 < nsteps ? (MODE_RELAX | MODE_MOVE) : MODE_RELAX;
        if ((s = launch_cell(ctx, P.B, P.prec, P.dim, P.xb, P.max_nb, P.first, P.top, st))) return s;
        if ((s = launch_fields(ctx, P.B, 0, st))) return s;
        if ((s = launch_ctl(ctx, P.B, 1, st))) return s;
    }
    return USP_OK;
}

usp_status ensure_side(usp_ctx* ctx, size_t n)
{
    if (!ctx->fork) HIPCHK(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    while (ctx->side.size() < n) {
        hipStream_t s2 = nullptr;
        hipEvent_t e2 = nullptr;
        HIPCHK(ctx, hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        HIPCHK(ctx, hipEventCreateWithFlags(&e2, hipEventDisableTiming));
        ctx->side.push_back(s2);
        ctx->join.push_back(e2);
    }
    return USP_OK;
}

// all groups: one group runs on the origin stream; several run side by side
// on their own streams, forked from and joined back to the origin
usp_status enqueue_all(usp_ctx* ctx, const std::vector<Plan>& plans, int nsteps, hipStream_t origin)
{
    if (plans.size() == 1) return enqueue_group(ctx, plans[0], nsteps, origin);
    usp_status s = ensure_side(ctx, plans.size());
    if (s) return s;
    HIPCHK(ctx, hipEventRecord(ctx->fork, origin));
    for (size_t i = 0; i < plans.size(); ++i) {
        HIPCHK(ctx, hipStreamWaitEvent(ctx->side[i], ctx->fork, 0));
        if ((s = enqueue_group(ctx, plans[i], nsteps, ctx->side[i]))) return s;
        HIPCHK(ctx, hipEventRecord(ctx->join[i], ctx->side[i]));
        HIPCHK(ctx, hipStreamWaitEvent(origin, ctx->join[i], 0));
    }
    return USP_OK;
}

}  // namespace

extern "C" {

usp_status usp_step(usp_ctx* ctx, const int* ids, int n_ids, int nsteps)
{
    if (!ctx || !ids || n_ids <= 0) return fail(ctx, USP_EINVAL, "no instances");
    if (nsteps <= 0) return USP_OK;
    std::vector<Plan> plans;
    usp_status s = make_plan(ctx, ids, n_ids, plans);
    if (s) return s;
    for (int i = 0; i < n_ids; ++i) {
        Instance* in = get_inst(ctx, ids[i]);
        in->sort_ok = in->h.diag != nullptr;
    }
    if (!ctx->graph || ctx->timing) return enqueue_all(ctx, plans, nsteps, ctx->stream);
    // graph mode: capture the whole call once, replay it afterwards
    std::vector<int> key(ids, ids + n_ids);
    key.push_back(-nsteps);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (!ctx->cap) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
        if (plans.size() > 1 && (s = ensure_side(ctx, plans.size()))) return s;
        HIPCHK(ctx, hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
        s = enqueue_all(ctx, plans, nsteps, ctx->cap);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(ctx->cap, &graph);
        if (s) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (ec != hipSuccess || !graph)
            return fail(ctx, USP_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess)
            return fail(ctx, USP_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
        it = ctx->graphs.emplace(key, exec).first;
    }
    HIPCHK(ctx, hipGraphLaunch(it->second, ctx->stream));
    return USP_OK;
}

usp_status usp_step_noalloc(usp_ctx* ctx, const int* ids, int n_ids, int nsteps)
{
    if (!ctx || !ids || n_ids <= 0) return fail(ctx, USP_EINVAL, "no instances");
    if (n_ids > NA_MAX_INST)
        return fail(ctx, USP_EINVAL, "usp_step_noalloc: more than 1024 instances in one call");
    if (!ctx->scratch) return fail(ctx, USP_EDEVICE, "usp_step_noalloc: no scratch address");
    // flavour of each instance; duplicates found after sorting by (flavour, id)
    long long key[NA_MAX_INST];
    long long cells = 0;
    for (int i = 0; i < n_ids; ++i) {
        Instance* in = get_inst(ctx, ids[i]);
        if (!in) return fail(ctx, USP_ESTATE, "unknown or freed instance in step");
        cells += in->h.ncell;
        const long long fl = ((((long long)(in->h.prec == 64) * 2 + (in->h.dim - 1)) * 2 +
                               in->xb()) * NSHAPE + in->first_shape()) * NSHAPE + in->top();
        key[i] = (fl << 32) | (long long)(uint32_t)ids[i];
    }
    if (cells > NA_MAX_CELLS)
        return fail(ctx, USP_EINVAL,
                    "usp_step_noalloc: more than 524288 cells in one call (" +
                        std::to_string(cells) + ")");
    std::sort(key, key + n_ids);
    for (int i = 1; i < n_ids; ++i)
        if (key[i] == key[i - 1])
            return fail(ctx, USP_EINVAL, "an instance listed twice in one step");
    if (nsteps <= 0) return USP_OK;
    InstDev* table = (InstDev*)ctx->scratch;
    int* base_all = (int*)((char*)ctx->scratch + NA_TABLE_BYTES);
    int* tiers = (int*)((char*)ctx->scratch + NA_TABLE_BYTES + NA_BASE_BYTES);
    // no timing events (they would be created here)
    const bool timing = ctx->timing;
    ctx->timing = false;
    auto run = [&]() -> usp_status {
        // one group per flavour, one after another on the context's stream;
        // the groups share the tier lists
        int g0 = 0, ngroup = 0;
        while (g0 < n_ids) {
            int g1 = g0;
            while (g1 < n_ids && (key[g1] >> 32) == (key[g0] >> 32)) ++g1;
            Instance* f = get_inst(ctx, (int)(uint32_t)key[g0]);
            int ncells = 0, max_nb = 0;
            for (int k = g0; k < g1; ++k) {
                const Instance* in = get_inst(ctx, (int)(uint32_t)key[k]);
                ncells += in->h.ncell;
                max_nb = std::max(max_nb, in->h.nb);
            }
            InstDev* tbl = table + g0;
            int* base = base_all + g0 + ngroup;
            for (int k = g0; k < g1; k += NA_PACK) {
                DescPack pk;
                pk.n = std::min(NA_PACK, g1 - k);
                for (int j = 0; j < pk.n; ++j) pk.src[j] = get_inst(ctx, (int)(uint32_t)key[k + j])->d;
                hipLaunchKernelGGL(na_copy_desc, dim3(pk.n), dim3(64), 0, ctx->stream, pk,
                                   tbl + (k - g0));
                HIPCHK(ctx, hipGetLastError());
            }
            hipLaunchKernelGGL(na_base_tiers, dim3(1), dim3(64), 0, ctx->stream, tbl, g1 - g0,
                               base, tiers, 1 + ncells);
            HIPCHK(ctx, hipGetLastError());
            Plan P;
            P.B.inst = tbl;
            P.B.base = base;
            P.B.ninst = g1 - g0;
            P.B.ncells = ncells;
            P.B.tiers = tiers;
            P.B.tier_stride = 1 + ncells;
            P.prec = f->h.prec;
            P.dim = f->h.dim;
            P.xb = f->xb();
            P.max_nb = max_nb;
            P.first = f->first_shape();
            P.top = f->top();
            usp_status st = prepare_cell(ctx, P.prec, P.dim, P.xb, max_nb, P.first, P.top);
            if (st) return st;
            if ((st = enqueue_group(ctx, P, nsteps, ctx->stream))) return st;
            g0 = g1;
            ++ngroup;
        }
        return USP_OK;
    };
    const usp_status s = run();
    ctx->timing = timing;
    if (s) return s;
    for (int i = 0; i < n_ids; ++i) {
        Instance* in = get_inst(ctx, ids[i]);
        in->sort_ok = in->h.diag != nullptr;
    }
    return USP_OK;
}

usp_status usp_set_shape(usp_ctx* ctx, int id, int first)
{
    Instance* in = get_inst(ctx, id);
    if (!in) return fail(ctx, USP_ESTATE, "unknown or freed instance");
    if (first < -1 || first >= NSHAPE || (first > in->top() && first < NSHAPE_WG))
        return fail(ctx, USP_EINVAL,
                    "first shape must be -1, a workgroup shape up to the instance's last, or "
                    "a wave shape");
    if (first == SHAPE_W6 && in->xb())
        return fail(ctx, USP_EINVAL,
                    "the 6-slot wave shape serves instances without open faces or the plate");
    if (first != in->first) {
        drop_groups(ctx);
        in->first = first;
    }
    return USP_OK;
}

usp_status usp_get_shape(usp_ctx* ctx, int id, int* first, int* last, int* nshape)
{
    Instance* in = get_inst(ctx, id);
    if (!in) return fail(ctx, USP_ESTATE, "unknown or freed instance");
    if (!first || !last || !nshape) return fail(ctx, USP_EINVAL, "null output");
    *first = in->first_shape();
    *last = in->top();
    *nshape = NSHAPE;
    return USP_OK;
}

usp_status usp_set_graph(usp_ctx* ctx, int on)
{
    if (!ctx) return USP_EINVAL;
    ctx->graph = on != 0;
    return USP_OK;
}

usp_status usp_sync(usp_ctx* ctx)
{
    if (!ctx) return USP_EINVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (size_t i = 0; i < ctx->inst.size(); ++i) {
        Instance* in = ctx->inst[i];
        if (!in || !in->alive) continue;
        int ctl[CTL_N];
        usp_status s = read_ctl(ctx, in, ctl);
        if (s) return s;
        if (ctl[CTL_ERR]) return err_status(ctx, ctl[CTL_ERR]);
    }
    return USP_OK;
}

usp_status usp_instance_status(usp_ctx* ctx, int id)
{
    Instance* in = get_inst(ctx, id);
    if (!in) return fail(ctx, USP_ESTATE, "unknown instance");
    int ctl[CTL_N];
    usp_status s = read_ctl(ctx, in, ctl);
    if (s) return s;
    return err_status(ctx, ctl[CTL_ERR]);
}

usp_status usp_num_cells(usp_ctx* ctx, int id, int* ncell)
{
    Instance* in = get_inst(ctx, id);
    if (!in || !ncell) return fail(ctx, USP_ESTATE, "unknown instance");
    *ncell = in->h.ncell;
    return USP_OK;
}

usp_status usp_num_particles(usp_ctx* ctx, int id, long long* n)
{
    Instance* in = get_inst(ctx, id);
    if (!in || !n) return fail(ctx, USP_ESTATE, "unknown instance");
    std::vector<int> cnt(in->h.ncell);
    HIPCHK(ctx, hipMemcpyAsync(cnt.data(), in->h.cnt, sizeof(int) * cnt.size(),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    long long t = 0;
    for (int c : cnt) t += c;
    *n = t;
    return USP_OK;
}

usp_status usp_get_state(usp_ctx* ctx, int id, int* counts, double* parts, double* cells,
                         int* step, int* n_samples)
{
    Instance* in = get_inst(ctx, id);
    if (!in) return fail(ctx, USP_ESTATE, "unknown instance");
    const InstDev& h = in->h;
    int ctl[CTL_N];
    usp_status s = read_ctl(ctx, in, ctl);
    if (s) return s;
    const int cur = ctl[CTL_CUR];
    const size_t ncell = (size_t)h.ncell, nb1 = (size_t)h.nb + 1;
    std::vector<uint32_t> tab(ncell * nb1);
    HIPCHK(ctx, hipMemcpy(tab.data(), h.tab[cur], tab.size() * 4, hipMemcpyDeviceToHost));
    if (counts)
        for (size_t c = 0; c < ncell; ++c) counts[c] = (int)tab[c * nb1 + h.nb];
    if (parts) {
        const size_t rb = h.prec == 32 ? 4 : 8;
        std::vector<unsigned char> buf(ncell * h.cap * rb);
        long long k0 = 0;
        std::vector<long long> off(ncell + 1, 0);
        for (size_t c = 0; c < ncell; ++c) off[c + 1] = off[c] + tab[c * nb1 + h.nb];
        for (int comp = 0; comp < 6; ++comp) {
            if (!h.pc[cur][comp]) {
                for (long long i = 0; i < off[ncell]; ++i) parts[6 * i + comp] = 0.0;
                continue;
            }
            HIPCHK(ctx, hipMemcpy(buf.data(), h.pc[cur][comp], buf.size(), hipMemcpyDeviceToHost));
            for (size_t c = 0; c < ncell; ++c) {
                const long long n = off[c + 1] - off[c];
                for (long long j = 0; j < n; ++j) {
                    const size_t src = c * h.cap + j;
                    const double v = h.prec == 32 ? (double)((float*)buf.data())[src]
                                                  : ((double*)buf.data())[src];
                    parts[6 * (off[c] + j) + comp] = v;
                }
            }
        }
        (void)k0;
    }
    if (cells) {
        std::vector<double> a(NMOM * ncell);
        double* arrs[4] = {h.mom, h.raw, h.avg, h.avgs};
        for (int q = 0; q < 4; ++q) {
            HIPCHK(ctx, hipMemcpy(a.data(), arrs[q], a.size() * 8, hipMemcpyDeviceToHost));
            for (size_t c = 0; c < ncell; ++c)
                for (int k = 0; k < NMOM; ++k) cells[c * (4 * NMOM + 2) + q * NMOM + k] = a[k * ncell + c];
        }
        std::vector<double> p(ncell);
        HIPCHK(ctx, hipMemcpy(p.data(), h.pcur, ncell * 8, hipMemcpyDeviceToHost));
        for (size_t c = 0; c < ncell; ++c) cells[c * (4 * NMOM + 2) + 4 * NMOM] = p[c];
        HIPCHK(ctx, hipMemcpy(p.data(), h.pprev, ncell * 8, hipMemcpyDeviceToHost));
        for (size_t c = 0; c < ncell; ++c) cells[c * (4 * NMOM + 2) + 4 * NMOM + 1] = p[c];
    }
    if (step) *step = ctl[CTL_STEP];
    if (n_samples) *n_samples = ctl[CTL_NSAMP];
    return err_status(ctx, ctl[CTL_ERR]);
}

usp_status usp_set_state(usp_ctx* ctx, int id, const int* counts, const double* parts,
                         const double* cells, int step, int n_samples)
{
    Instance* in = get_inst(ctx, id);
    if (!in || !counts || !parts) return fail(ctx, USP_EINVAL, "bad set_state arguments");
    if (step < 0 || n_samples < 0)
        return fail(ctx, USP_EINVAL, "step and n_samples must be non-negative");
    const InstDev& h = in->h;
    in->sort_ok = false;
    int ctl[CTL_N];
    usp_status s = read_ctl(ctx, in, ctl);
    if (s) return s;
    const int cur = ctl[CTL_CUR];
    const size_t ncell = (size_t)h.ncell, nb1 = (size_t)h.nb + 1;
    for (size_t c = 0; c < ncell; ++c)
        if (counts[c] < 0 || counts[c] > h.max_ppc)
            return fail(ctx, USP_ECAPACITY, "a cell holds more than max_ppc particles");
    std::vector<long long> off(ncell + 1, 0);
    for (size_t c = 0; c < ncell; ++c) off[c + 1] = off[c] + counts[c];
    const size_t rb = h.prec == 32 ? 4 : 8;
    std::vector<unsigned char> buf(ncell * h.cap * rb, 0);
    for (int comp = 0; comp < 6; ++comp) {
        if (!h.pc[cur][comp]) continue;
        for (size_t c = 0; c < ncell; ++c)
            for (long long j = 0; j < counts[c]; ++j) {
                const double v = parts[6 * (off[c] + j) + comp];
                const size_t dst = c * h.cap + j;
                if (h.prec == 32) ((float*)buf.data())[dst] = (float)v;
                else ((double*)buf.data())[dst] = v;
            }
        HIPCHK(ctx, hipMemcpy(h.pc[cur][comp], buf.data(), buf.size(), hipMemcpyHostToDevice));
    }
    std::vector<uint32_t> tab(ncell * nb1);
    const int centre = h.Ky * h.nbx + h.Kx;
    for (size_t c = 0; c < ncell; ++c)
        for (int b = 0; b <= h.nb; ++b) tab[c * nb1 + b] = b <= centre ? 0u : (uint32_t)counts[c];
    HIPCHK(ctx, hipMemcpy(h.tab[cur], tab.data(), tab.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(h.cnt, counts, ncell * 4, hipMemcpyHostToDevice));
    int nctl[CTL_N] = {cur, step, cells ? n_samples : 0, 0};
    HIPCHK(ctx, hipMemcpy(h.ctl, nctl, sizeof(nctl), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemset(h.far_n, 0, 2 * sizeof(int)));
    if (cells) {
        std::vector<double> a(NMOM * ncell);
        double* arrs[4] = {h.mom, h.raw, h.avg, h.avgs};
        for (int q = 0; q < 4; ++q) {
            for (size_t c = 0; c < ncell; ++c)
                for (int k = 0; k < NMOM; ++k) a[k * ncell + c] = cells[c * (4 * NMOM + 2) + q * NMOM + k];
            HIPCHK(ctx, hipMemcpy(arrs[q], a.data(), a.size() * 8, hipMemcpyHostToDevice));
        }
        std::vector<double> p(ncell);
        for (size_t c = 0; c < ncell; ++c) p[c] = cells[c * (4 * NMOM + 2) + 4 * NMOM];
        HIPCHK(ctx, hipMemcpy(h.pcur, p.data(), ncell * 8, hipMemcpyHostToDevice));
        for (size_t c = 0; c < ncell; ++c) p[c] = cells[c * (4 * NMOM + 2) + 4 * NMOM + 1];
        HIPCHK(ctx, hipMemcpy(h.pprev, p.data(), ncell * 8, hipMemcpyHostToDevice));
        return USP_OK;
    }
    HIPCHK(ctx, hipMemset(h.avg, 0, NMOM * ncell * 8));
    HIPCHK(ctx, hipMemset(h.avgs, 0, NMOM * ncell * 8));
    if ((s = finish_state(ctx, in))) return s;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return USP_OK;
}

usp_status usp_get_fields(usp_ctx* ctx, int id, int which, double* out)
{
    Instance* in = get_inst(ctx, id);
    if (!in || !out) return fail(ctx, USP_EINVAL, "bad get_fields arguments");
    const size_t ncell = (size_t)in->h.ncell;
    double* d = nullptr;
    HIPCHK(ctx, hipMalloc(&d, ncell * 18 * 8));
    Batch B = single_batch(in, 0);
    hipLaunchKernelGGL(fields_out_kernel, dim3((ncell + 255) / 256), dim3(256), 0, ctx->stream, B,
                       which, d, 0);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipMemcpyAsync(out, d, ncell * 18 * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(d);
    return USP_OK;
}

usp_status usp_moments(usp_ctx* ctx, int id, int which, usp_moments_view* out)
{
    Instance* in = get_inst(ctx, id);
    if (!in || !out || (which != 0 && which != 1))
        return fail(ctx, USP_EINVAL, "bad moments arguments");
    const size_t ncell = (size_t)in->h.ncell;
    if (!in->fview) {
        in->fview = (double*)dalloc(ctx, ncell * 18 * 8);
        if (!in->fview) return fail(ctx, USP_ENOMEM, "moments view");
        in->allocs.push_back(in->fview);
        in->bytes += ncell * 18 * 8;
    }
    Batch B = single_batch(in, 0);
    hipLaunchKernelGGL(fields_out_kernel, dim3((ncell + 255) / 256), dim3(256), 0, ctx->stream, B,
                       which, in->fview, 1);
    HIPCHK(ctx, hipGetLastError());
    out->ncell = (int)ncell;
    out->nfield = 18;
    out->data = in->fview;
    return USP_OK;
}

usp_status usp_set_diag(usp_ctx* ctx, int id, int on)
{
    Instance* in = get_inst(ctx, id);
    if (!in) return fail(ctx, USP_ESTATE, "unknown instance");
    in->sort_ok = false;
    if (on && !in->h.diag) {
        if (!in->dg_mem) {
            const size_t slots = (size_t)in->h.ncell * in->h.cap;
            auto A = [&](size_t bytes) -> void* {
                void* p = dalloc(ctx, bytes);
                if (p) {
                    in->allocs.push_back(p);
                    in->bytes += bytes;
                }
                return p;
            };
            in->dg_mem = (double*)A((size_t)in->h.ncell * NDIAG * 8);
            in->ori_mem[0] = (uint32_t*)A(slots * 4);
            in->ori_mem[1] = (uint32_t*)A(slots * 4);
            in->sorg_mem = (uint64_t*)A(slots * 8);
            if (!in->dg_mem || !in->ori_mem[0] || !in->ori_mem[1] || !in->sorg_mem)
                return fail(ctx, USP_ENOMEM, "diag buffers");
        }
        HIPCHK(ctx, hipMemsetAsync(in->dg_mem, 0, (size_t)in->h.ncell * NDIAG * 8, ctx->stream));
        in->h.diag = in->dg_mem;
        in->h.ori[0] = in->ori_mem[0];
        in->h.ori[1] = in->ori_mem[1];
        in->h.sorg = in->sorg_mem;
    } else if (!on) {
        in->h.diag = nullptr;
        in->h.ori[0] = in->h.ori[1] = nullptr;
        in->h.sorg = nullptr;
    }
    drop_groups(ctx);
    return upload_desc(ctx, in);
}

usp_status usp_get_sort(usp_ctx* ctx, int id, int32_t* cell_offsets, int32_t* perm)
{
    Instance* in = get_inst(ctx, id);
    if (!in) return fail(ctx, USP_ESTATE, "unknown instance");
    if (!cell_offsets) return fail(ctx, USP_EINVAL, "null cell_offsets");
    if (!in->h.diag || !in->sort_ok)
        return fail(ctx, USP_ESTATE, "no step has run with diagnostics on since the last load");
    const size_t ncell = (size_t)in->h.ncell, cap = (size_t)in->h.cap;
    std::vector<double> dg(ncell * NDIAG);
    HIPCHK(ctx, hipMemcpyAsync(dg.data(), in->h.diag, dg.size() * 8, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<long long> pre(ncell + 1, 0);
    cell_offsets[0] = 0;
    for (size_t c = 0; c < ncell; ++c) {
        cell_offsets[c + 1] = cell_offsets[c] + (int32_t)dg[c * NDIAG + D_NIN];
        pre[c + 1] = pre[c] + (long long)dg[c * NDIAG + D_NPRE];
    }
    if (!perm) return USP_OK;
    std::vector<uint64_t> so(ncell * cap);
    HIPCHK(ctx, hipMemcpyAsync(so.data(), in->h.sorg, so.size() * 8, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (size_t c = 0; c < ncell; ++c) {
        const int n = cell_offsets[c + 1] - cell_offsets[c];
        for (int j = 0; j < n; ++j) {
            const uint64_t v = so[c * cap + j];
            const size_t src = (size_t)(v >> 32);
            if (src >= ncell) return fail(ctx, USP_ESTATE, "sort record out of range");
            perm[cell_offsets[c] + j] = (int32_t)(pre[src] + (long long)(v & 0xFFFFFFFFu));
        }
    }
    return USP_OK;
}

usp_status usp_stats(usp_ctx* ctx, int id, usp_stats_t* out)
{
    Instance* in = get_inst(ctx, id);
    if (!in) return fail(ctx, USP_ESTATE, "unknown instance");
    if (!out) return fail(ctx, USP_EINVAL, "null stats");
    memset(out, 0, sizeof(*out));
    int ctl[CTL_N];
    usp_status s = read_ctl(ctx, in, ctl);
    if (s) return s;
    const size_t ncell = (size_t)in->h.ncell;
    std::vector<int> cnt(ncell);
    HIPCHK(ctx, hipMemcpyAsync(cnt.data(), in->h.cnt, ncell * 4, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int c : cnt) out->live += c;
    out->step = ctl[CTL_STEP];
    out->error = ctl[CTL_ERR] ? (int)err_status(ctx, ctl[CTL_ERR]) : 0;
    out->diag = in->h.diag != nullptr && in->sort_ok;
    if (!out->diag) return USP_OK;
    std::vector<double> dg(ncell * NDIAG);
    HIPCHK(ctx, hipMemcpyAsync(dg.data(), in->h.diag, dg.size() * 8, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (size_t c = 0; c < ncell; ++c) {
        const double* d = dg.data() + c * NDIAG;
        out->added[0] += (long long)d[D_N2];
        out->added[1] += (long long)d[D_N4];
        out->added[2] += (long long)d[D_N7];
        out->selected += (long long)d[D_NSEL];
        out->reassigned += (long long)d[D_NUSP];
        out->deleted += (long long)d[D_NDEL];
        out->entered += (long long)d[D_NINJ];
        out->left += (long long)d[D_NGONE];
        out->clamped += (long long)d[D_CLAMP];
        out->es_fallback += (long long)d[D_CHOLFB];
        const int f = (int)d[D_FLAGS];
        out->cells_invalid += (f & F_SKIP) != 0;
        out->mass_fail += (f & F_FAILMASS) != 0;
        out->energy_fail += (f & F_FAILENERGY) != 0;
        out->whole_cell += (f & F_WHOLE) != 0;
    }
    return USP_OK;
}

usp_status usp_get_diag(usp_ctx* ctx, int id, double* out)
{
    Instance* in = get_inst(ctx, id);
    if (!in || !out || !in->h.diag) return fail(ctx, USP_ESTATE, "diagnostics not enabled");
    HIPCHK(ctx, hipMemcpyAsync(out, in->h.diag, (size_t)in->h.ncell * NDIAG * 8,
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return USP_OK;
}

usp_status usp_set_timing(usp_ctx* ctx, int on)
{
    if (!ctx) return USP_EINVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto& e : ctx->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    ctx->events.clear();
    ctx->timed_passes = 0;
    ctx->timing = on != 0;
    return USP_OK;
}

usp_status usp_get_timing(usp_ctx* ctx, double* ms, long long* passes)
{
    if (!ctx || !ms || !passes) return USP_EINVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    double t = 0.0;
    for (auto& e : ctx->events) {
        float f = 0.0f;
        HIPCHK(ctx, hipEventElapsedTime(&f, e.first, e.second));
        t += f;
    }
    *ms = t;
    *passes = ctx->timed_passes;
    return USP_OK;
}

usp_status usp_philox(usp_ctx* ctx, const uint32_t* ctr, uint32_t k0, uint32_t k1, int n,
                      uint32_t* out)
{
    if (!ctx || !ctr || !out || n <= 0) return USP_EINVAL;
    uint32_t *dc = nullptr, *dout = nullptr;
    HIPCHK(ctx, hipMalloc(&dc, (size_t)n * 16));
    HIPCHK(ctx, hipMalloc(&dout, (size_t)n * 16));
    HIPCHK(ctx, hipMemcpy(dc, ctr, (size_t)n * 16, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(philox_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, dc, k0, k1,
                       n, dout);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost));
    (void)hipFree(dc);
    (void)hipFree(dout);
    return USP_OK;
}

}  // extern "C"
