// Shared declarations of the libusp host runtime and its gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace usp {

constexpr int NMOM = 13;   // centred moments / raw sums per cell
constexpr int NDIAG = 48;  // per-cell diagnostic record
constexpr int NDIAG_STEP = 32;  // slots describing the last step; then phase cycle counters
constexpr int MAX_BINS = 256;
constexpr int MAX_PPC = 2048;

// LDS tables of the cell kernel that depend on the workgroup size: a cell
// held by one wave (64 threads, at most 512 particle slots) takes smaller
// ones than a cell held by 256 threads
struct LdsDims {
    int far;   // far arrivals one cell can take per step
    int psb;   // added particles per chunk of the batch-order Gram sums
    int kth;   // buckets of the rank-threshold histogram (top bits of the key)
    int nw;    // waves per workgroup
};
__host__ __device__ constexpr LdsDims lds_dims(int nt)
{
    return nt == 64 ? LdsDims{128, 64, 64, 1} : LdsDims{128, 256, 2048, 4};
}

// control words of an instance (device memory)
enum { CTL_CUR = 0, CTL_STEP = 1, CTL_NSAMP = 2, CTL_ERR = 3, CTL_N = 4 };
// sticky error bits
enum { ERR_CAPACITY = 1, ERR_WINDOW = 2, ERR_NONFINITE = 4 };

// kernel modes
enum {
    MODE_RELAX = 1,    // Table 2 steps 4-8 on the gathered cell
    MODE_MOVE = 2,     // step 2 + step 3 of the next step, write by destination bins
    MODE_MOMENTS = 4   // only the moments of the gathered cell (initial state)
};

// Philox purposes (counter word 1 = purpose << 24 | sub)
enum {
    PUR_INIT_POS = 1,
    PUR_INIT_VEL = 2,
    PUR_SPAWN_CNT = 3,
    PUR_SPAWN_POS = 4,
    PUR_SPAWN_VEL = 5,
    PUR_WALL = 6,
    PUR_SELECT = 7,
    PUR_RESAMPLE = 8,
    PUR_INJECT_CNT = 9,
    PUR_INJECT = 10,
    PUR_INJECT_POS = 11
};

// diagnostic slots (same meaning as the host-side record)
enum {
    D_NIN = 0, D_N4, D_NSEL, D_NUSP, D_NDEL, D_N7, D_NOUT, D_N2, D_SSEL, D_PSEL, D_FLAGS,
    D_CHOLFB, D_M0, D_P0X, D_P0Y, D_P0Z, D_E0, D_M1, D_P1X, D_P1Y, D_P1Z, D_E1, D_CLAMP,
    D_MARG_SEL, D_MARG_ROUND, D_MARG_CNT, D_WR, D_S2, D_MARG_CNT2, D_NINJ, D_NGONE,
    D_NPRE  // particles of the cell before the step-3 sort (present, step 2, entered)
};
enum { F_SKIP = 1, F_FAILMASS = 2, F_FAILENERGY = 4, F_NOUSP = 8, F_WHOLE = 16 };
// device-only diagnostic slot: particle slots of the shape that finished the cell
constexpr int D_SHAPE_SLOTS = 47;

// Everything a kernel needs to know about one solver instance.  Lives in
// device memory; read-only during a launch.
struct InstDev {
    // gas
    double m, kB, mu_ref, T_ref, omega, Pr, R, F;
    // geometry
    int dim, nx, ny, ncell;
    double x0, x1, y0, y1, dx, dy, inv_dx, inv_dy, vcell, Np;
    int face_kind[4];
    double face_T[4];
    double face_u[12];
    double accel[3];
    // open faces (kind 3): reservoir density, and the second chamber's state
    // beyond the split coordinate; bit f of open_mask set for an open face f
    double face_n[4], face_split[4], face_nb[4], face_Tb[4];
    int open_mask;
    // internal plate (2-D): thin diffuse wall on x = plate_x, plate_ylo <= y <= plate_yhi
    int plate;
    double plate_x, plate_ylo, plate_yhi, plate_T;
    // numerics
    double dt, r_p, Kn_c, pne_fixed;
    int pne_mode, n_avg, avg_start, prec, weight_mode, conserve_mode, max_ppc, jmom_mode, proj;
    int avg_init;
    int scheme;  // 0 USP-ESBGK, 1 SP-ESBGK (Table 1)
    int es_mode;  // 0 alpha(t) per particle (Eq. 29-32), 1 its expectation per cell
    int gll_u;    // Eq. 18 velocity term over 0 max(|u|, sound speed), 1 |u|
    int select_mode;  // step 5: 0 Bernoulli trial per particle, 1 Eq. 9 count
    int es_sampler;   // step 6: 0 Cholesky factor of f_G(t), 1 Eq. 11 linear map
    uint32_t key0, key1;
    // sort window: source offsets -Kx..Kx, -Ky..Ky; nb = (2Ky+1)(2Kx+1) bins
    int Kx, Ky, nbx, nb;
    int cap;  // particle slots per cell region (>= max_ppc)
    // device arrays
    void* pc[2][6];     // [buffer][x, y, cx, cy, cz, w]
    uint32_t* tab[2];   // [buffer][cell][nb + 1] exclusive bin offsets
    double* mom;        // [NMOM][ncell] centred moments of f^n
    double* raw;        // [NMOM][ncell] raw sums of f^n
    double* avg;        // [NMOM][ncell] Eq. 34 average of raw sums of f^n
    double* avgs;       // [NMOM][ncell] Eq. 34 average of raw sums of f-tilde^*
    double* pcur;       // [ncell] P_ne^n
    double* pprev;      // [ncell] P_ne^{n-1}
    int* cnt;           // [ncell] particles of f^n per cell
    int* ctl;           // [CTL_N]
    double* diag;       // [ncell][NDIAG] or null
    // with diagnostics: the logical slot each stored particle had when it
    // was moved (per buffer), and the origin (source cell << 32 | slot) of
    // every particle of f-tilde^* as gathered (the record of the sort)
    uint32_t* ori[2];
    uint64_t* sorg;
    // particles displaced beyond the window: per buffer a list of
    // (destination cell, source offset key, slot) + the particle, and a count
    int far_cap;
    int* far_n;         // [2]
    uint32_t* far_meta[2];  // [far_cap][3]
    void* far_pc[2][6];
};

struct Batch {
    const InstDev* inst;  // [ninst]
    const int* base;      // [ninst + 1] first global cell of each instance
    int ninst;
    int ncells;           // total cells
    int mode;
    // per-cell shape tiers: a launch of a small shape hands cells that need
    // more particle slots to the next shape.  Each list is [count, cells...].
    int* tiers = nullptr;           // NSHAPE lists of tier_stride ints (counts cleared by ctl_kernel)
    int tier_stride = 0;
    const int* tier_in = nullptr;   // cells of this launch (null: every cell)
    int* tier_out = nullptr;        // cells handed on (null: last shape, overflow is an error)
};

// LDS bytes of the cell kernel of `nt` threads for `cap` particle slots and
// `nb` bins (the same carving as the kernel: every array rounded up to 16
// bytes)
inline size_t lds_bytes(int nt, int cap, int nb)
{
    auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
    const LdsDims d = lds_dims(nt);
    size_t b = 0;
    b += r16((size_t)cap * 4);                  // gather map
    b += r16((size_t)(cap / 64) * nb * 2);      // bin tile counts
    b += r16((size_t)d.kth * 4) + r16(64 * 4);  // histogram, scan totals
    b += r16((size_t)d.nw * 24 * 8);            // reductions (one row per wave)
    b += 4 * r16((size_t)(nb + 1) * 4);         // runs, bin offsets
    b += r16((size_t)d.far * 8) + 3 * r16((size_t)d.far * 4) + r16(16);  // far arrivals
    b += r16(64 * 8);                           // scalars
    b += r16((size_t)d.psb * 6 * 8);            // Gram-sum staging
    b += r16(32 * 8);                           // pending moments
    b += r16(48 * 8);                           // per-cell inputs
    b += r16(16 * 8);                           // phase time stamps
    b += r16(256) + r16(32 * 8);                // cell scalars, moments
    return b;
}

// Launch shapes of the cell kernel (threads per cell, particle slots per
// thread).  Slot columns beyond a cell's count are skipped at run time, so a
// larger shape costs registers and LDS, not instructions.
//
// Two families.  The workgroup shapes (0..4) hold a cell in 256 threads:
// particle j always sits in thread j mod 256, so every reduction adds the
// same numbers in the same order whatever workgroup shape runs a cell.  6
// slots per thread is the most that fits the registers at two workgroups per
// CU; the 8-slot shape (it spills) serves the rare cells of more than 1536
// particles.  The wave shapes (5, 6) hold a cell in one wave of 64 threads
// (particle j in lane j mod 64) with 4 or 6 slots per lane: a CU keeps 16
// cells in flight instead of 4, and a cell's phases need no barrier between
// waves, which is what cells of a few hundred particles are bound by.  Wave
// shapes agree with each other bit for bit, not with the workgroup shapes
// (their sums run in another order), so an instance keeps its family.  The
// 6-slot wave shape serves instances without open faces or the plate only.
struct Shape {
    int nt, ppt, ppt2;  // ppt2 > 0: cells that need more than nt x ppt slots rerun with ppt2
    int slots() const { return nt * (ppt2 > ppt ? ppt2 : ppt); }
};
constexpr int NSHAPE = 7;
constexpr int NSHAPE_WG = 5;  // workgroup shapes; the wave shapes follow
constexpr Shape SHAPES[NSHAPE] = {{256, 1, 0}, {256, 2, 0}, {256, 4, 0}, {256, 4, 6},
                                  {256, 8, 0}, {64, 4, 0},  {64, 6, 0}};
constexpr int SHAPE_W4 = 5, SHAPE_W6 = 6;
// the last shape of an instance: the smallest workgroup shape that holds
// max_ppc particles and the step-2 particles of a full cell
inline int pick_shape_index(int max_ppc)
{
    const int need = max_ppc + max_ppc / 8 + 1;
    for (int i = 0; i + 1 < NSHAPE_WG; ++i)
        if (need <= SHAPES[i].slots()) return i;
    return NSHAPE_WG - 1;
}
inline Shape pick_shape(int max_ppc) { return SHAPES[pick_shape_index(max_ppc)]; }
// the first launch shape of an instance that needs the largest one
constexpr int TIER_FIRST = 3;
// The launches of one pass: the first shape, then every workgroup shape up
// to the last that holds more slots than the shape before it (a cell is
// handed on only to a shape that can hold more).  Returns the count.
inline int shape_chain(int first, int top, int* out)
{
    int n = 0;
    out[n++] = first;
    int slots = SHAPES[first].slots();
    for (int t = 0; t <= top && t < NSHAPE_WG; ++t)
        if (t != first && SHAPES[t].slots() > slots) {
            out[n++] = t;
            slots = SHAPES[t].slots();
        }
    return n;
}

}  // namespace usp
