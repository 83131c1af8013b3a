// gfx950 cell kernel of the USP-ESBGK time step (arXiv 1808.03801, Table 2).
//
// One workgroup of NT threads owns one cell: 256 threads (four waves) for
// the workgroup shapes, one wave of 64 threads for the wave shapes.  The
// cell's particles live in registers: particle j of the cell is held by
// thread j % NT in register slot j / NT (PPT slots per thread, fully
// unrolled), so every per-particle phase runs without LDS traffic and with
// PPT independent instruction streams per thread.  LDS holds only tables:
// the gather map, bin tile counts, the rank histogram, reduction scratch, the
// staging of the Gram sums of added batches and the cell scalars.  PPT is a
// template parameter (1, 2, 4, 6 or 8); the 4|6 kernel reruns a cell that
// needs more than 1024 slots with 6 per thread in the same workgroup.  A
// one-wave cell synchronises its lanes through LDS alone (no barrier).
//
// Phases for one cell (mode bits select them):
//   gather    read the cell's arrivals from the neighbours' bins in canonical
//             order (source offset, then source slot), far movers merged in;
//   relax     Eq. 33 moments, step 4 (added particles for f^*), step 5
//             (Bernoulli selection, keep int(sum W) with the smallest keys),
//             step 6 (f_G(t) resampling), step 7 (added particles), the
//             conservation correction, step 8 moments and Eq. 34 averages;
//   move      step 2 of the next time level, step 3 (advect, walls), and the
//             write-out grouped by destination offset with a bin table;
//   stay      (no move) write the cell's particles back in slot order.
//
// Particles removed in step 5 are not moved out of their registers: their
// fate marks them dead, and the logical slot of each survivor comes from a
// scan.  Physical order is monotone in logical order, so stable ranks taken
// over physical positions equal those over logical slots.
#pragma once

#include "usp_device.h"

namespace usp {

constexpr int FAR_BIN = 0xFFFF;
constexpr uint32_t FAR_PENDING = 0xFFFEu;  // leaves the sort window; far list not yet written
constexpr uint32_t FARBIT = 0x80000000u;

// fate codes
enum { FT_KEEP = 0, FT_REASSIGN = 1, FT_DELETE = 2, FT_SEL = 3, FT_EMPTY = 4 };

struct Lds {
    uint32_t* srcmap;  // [cap] source index of each gathered position
    uint16_t* tiles;   // [cap / 64][nb]
    uint32_t* hist;    // [lds_dims(NT).kth]
    uint32_t* wtot;    // [64] per-wave scan totals
    double* red;       // [NW][24]
    uint32_t* run_pre;
    uint32_t* run_src;
    uint32_t* run_dst;
    uint32_t* boff;
    uint64_t* fkey;
    uint32_t* fent;
    uint32_t* fpos;
    uint32_t* fib;
    uint32_t* fcount;
    double* sc;
    double* psb;   // [psb][6] basis values and weight of added particles (Gram sums)
    CellF* f;      // cell scalars shared by the workgroup
    double* mom;   // [0..12] centred, [13..25] averages, [26] energy, [27..29] momentum
    double* pend;  // [0..12] raw sums, [13..25] J-moment averages, [26] count: stored
                   // to HBM once the cell can no longer be handed to a larger shape
    long long* tst;  // [16] phase time stamps (diagnostics), [15] = start
    double* pre;   // per-cell inputs loaded at the start: [0..12] J-moment averages,
                   // [13..25] Eq. 34 averages, [26..38] moments, [39] P_ne^n, [40] P_ne^n-1
};

static_assert(sizeof(CellF) <= 256, "cell scalars must fit their LDS slot");

template <int NT>
__device__ __forceinline__ Lds carve(unsigned char* sm, int cap, int nb)
{
    constexpr LdsDims D = lds_dims(NT);
    Lds L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        unsigned char* q = sm + o;
        o += (bytes + 15) & ~(size_t)15;
        return q;
    };
    L.srcmap = (uint32_t*)take((size_t)cap * 4);
    L.tiles = (uint16_t*)take((size_t)(cap / 64) * nb * 2);
    L.hist = (uint32_t*)take((size_t)D.kth * 4);
    L.wtot = (uint32_t*)take(64 * 4);
    L.red = (double*)take((size_t)D.nw * 24 * 8);
    L.run_pre = (uint32_t*)take((size_t)(nb + 1) * 4);
    L.run_src = (uint32_t*)take((size_t)(nb + 1) * 4);
    L.run_dst = (uint32_t*)take((size_t)(nb + 1) * 4);
    L.boff = (uint32_t*)take((size_t)(nb + 1) * 4);
    L.fkey = (uint64_t*)take((size_t)D.far * 8);
    L.fent = (uint32_t*)take((size_t)D.far * 4);
    L.fpos = (uint32_t*)take((size_t)D.far * 4);
    L.fib = (uint32_t*)take((size_t)D.far * 4);
    L.fcount = (uint32_t*)take(16);
    L.sc = (double*)take(64 * 8);
    L.psb = (double*)take((size_t)D.psb * 6 * 8);
    L.f = (CellF*)take(sizeof(CellF));
    L.mom = (double*)take(32 * 8);
    L.pend = (double*)take(32 * 8);
    L.pre = (double*)take(48 * 8);
    L.tst = (long long*)take(16 * 8);
    return L;
}

// a value known to be equal in all lanes, made visibly uniform (scalar)
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Make the workgroup's LDS writes visible to all its threads.  A one-wave
// workgroup runs its lanes in lock step, so completing its own LDS
// operations (and keeping the compiler from moving LDS accesses across) is
// enough; larger workgroups need the barrier.
template <int NT>
__device__ __forceinline__ void wg_sync()
{
    if constexpr (NT == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    } else {
        __syncthreads();
    }
}

template <int NT, int K>
__device__ __forceinline__ void bsum(double (&v)[K], double* red, int tid)
{
    constexpr int NW = NT / 64;
    if constexpr (K >= 4) {
        wave_sums<K>(v);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    }
    if constexpr (NW == 1) return;  // one wave: every lane holds the total
    const int lane = tid & 63, wave = tid >> 6;
    wg_sync<NT>();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
    wg_sync<NT>();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += red[w * K + k];
        v[k] = s;
    }
}

template <int NT>
__device__ __forceinline__ double bmin(double v, double* red, int tid)
{
    constexpr int NW = NT / 64;
    v = wave_min(v);
    if constexpr (NW == 1) return v;
    const int lane = tid & 63, wave = tid >> 6;
    wg_sync<NT>();
    if (lane == 0) red[wave] = v;
    wg_sync<NT>();
    double m = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) m = fmin(m, red[w]);
    return m;
}

// exclusive prefix of flag over physical positions j = k * NT + tid
template <int NT, int PPT>
__device__ __forceinline__ int phys_scan(const bool (&flag)[PPT], int (&pre)[PPT], uint32_t* wtot,
                                         int tid)
{
    constexpr int NW = NT / 64;
    const int lane = tid & 63, wave = tid >> 6;
    if constexpr (NW == 1) {
        int base = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const uint64_t m = __ballot(flag[k]);
            pre[k] = base + __popcll(m & lanemask_lt(lane));
            base += __popcll(m);
        }
        return base;
    }
    int wpre[PPT];
    wg_sync<NT>();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint64_t m = __ballot(flag[k]);
        wpre[k] = __popcll(m & lanemask_lt(lane));
        if (lane == 0) wtot[k * NW + wave] = (uint32_t)__popcll(m);
    }
    wg_sync<NT>();
    int base = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        int off = base, tot = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int t = (int)wtot[k * NW + w];
            if (w < wave) off += t;
            tot += t;
        }
        pre[k] = off + wpre[k];
        base += tot;
    }
    return base;
}

// exclusive scan of up to 256 counters in place by the first wave; a[n] = total
__device__ __forceinline__ void wave0_scan(uint32_t* a, int n, int tid)
{
    if (tid < 64) {
        uint32_t loc[4], s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = 4 * tid + q;
            loc[q] = b < n ? a[b] : 0u;
            s += loc[q];
        }
        uint32_t incl = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, 64);
            if (tid >= o) incl += t;
        }
        uint32_t run = incl - s;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = 4 * tid + q;
            if (b < n) a[b] = run;
            run += loc[q];
        }
        if (tid == 63) a[n] = incl;
    }
}

template <typename real, int DIM, int PPT>
struct Parts {
    real x[DIM == 2 ? PPT : 1];
    real y[PPT], c0[PPT], c1[PPT], c2[PPT], w[PPT];
    uint32_t key[PPT];  // rank key (relax), bin / output position (move)
    uint32_t st[PPT];   // fate | logical slot << 8
};

template <typename real, int DIM, int PPT>
__device__ __forceinline__ int fate(const Parts<real, DIM, PPT>& P, int k)
{
    return (int)(P.st[k] & 0xFFu);
}

// ---------------------------------------------------------------------------
// moments of the live particles (fate keep or reassigned): raw sums in one
// pass, centred from them; E = sum w |c|^2 / 2.  Every thread gets the results.
// ---------------------------------------------------------------------------
template <int NT, typename real, int DIM, int PPT>
__device__ __forceinline__ void moments_r(const Parts<real, DIM, PPT>& P, const Lds& L, int tid,
                                          int nuse, double* cen, double* raw, double* E)
{
    double a[14];
#pragma unroll
    for (int q = 0; q < 14; ++q) a[q] = 0.0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (k * NT < nuse && fate(P, k) <= FT_REASSIGN) {
            const double w = (double)P.w[k];
            const double c0 = (double)P.c0[k], c1 = (double)P.c1[k], c2 = (double)P.c2[k];
            const double cc = c0 * c0 + c1 * c1 + c2 * c2;
            a[0] += w;
            a[1] += w * c0;
            a[2] += w * c1;
            a[3] += w * c2;
            a[4] += 0.5 * w * cc;
            a[5] += w * c0 * c0;
            a[6] += w * c1 * c1;
            a[7] += w * c2 * c2;
            a[8] += w * c0 * c1;
            a[9] += w * c0 * c2;
            a[10] += w * c1 * c2;
            a[11] += w * cc * c0;
            a[12] += w * cc * c1;
            a[13] += w * cc * c2;
        }
    }
    bsum<NT>(a, L.red, tid);
    // centred moments from the raw sums (FP64: the cancellation costs
    // (|u|^2 / theta) of the 53 bits, far below the state precision)
    *E = a[4];
    raw[0] = a[0];
#pragma unroll
    for (int q = 0; q < 3; ++q) raw[1 + q] = a[1 + q];
#pragma unroll
    for (int q = 0; q < 9; ++q) raw[4 + q] = a[5 + q];
    centred_from_raw(raw, cen);
}

// ---------------------------------------------------------------------------
// Added particles of batch 2, 4 or 7 (Eq. 25-27, Table 2) at physical
// positions [a, a + n) with logical slots [ls, ls + n).  Sampling in double
// precision, stored once rounded.  Optional zero-moment projection.
// ---------------------------------------------------------------------------
// Eq. 25 count of an added batch: S0 min(1, x) / r_p rounded
// stochastically (floor plus a Bernoulli draw of the fraction); 0 for an
// invalid cell or P_ne = 0.  `marg` (optional) keeps the smallest distance
// of the draw from its threshold.
__device__ __forceinline__ int spawn_count(const InstDev& I, int batch, int cell, uint32_t step,
                                           const CellF& f, double pne, double* marg)
{
    if (!f.valid || !(pne > 0.0) || !(f.x > 0.0)) return 0;
    const double m1 = f.x < 1.0 ? f.x : 1.0;
    // held in [0, 1e6] before it becomes an int: a blown-up cell's S0 must
    // reach the capacity tests, not overflow the int (a count of 2^31 wraps
    // the capacity sums negative)
    const double v = fmin(fmax(f.S0 * m1 / I.r_p, 0.0), 1.0e6);
    uint32_t r[4];
    draw(I, step, PUR_SPAWN_CNT, (uint32_t)batch, (uint32_t)cell, 0u, r);
    const double u = uni_d(r[0], I.prec);
    const double fl = floor(v);
    if (marg) *marg = fmin(*marg, fabs(u - (v - fl)));
    return (int)fl + (u < v - fl ? 1 : 0);
}

template <int NT, typename real, int DIM, int PPT>
__device__ __forceinline__ int spawn_r(const InstDev& I, Parts<real, DIM, PPT>& P, const Lds& L,
                                       int batch, int cell, int ix, int iy, uint32_t step,
                                       const CellF& f, double pne, int a, int ls, int tid,
                                       uint32_t* errbits, double* marg, bool can_defer)
{
    if (!f.valid || !(pne > 0.0) || !(f.x > 0.0)) return 0;
    const double m1 = f.x < 1.0 ? f.x : 1.0;
    int na = spawn_count(I, batch, cell, step, f, pne, marg);
    if (ls + na > I.max_ppc || a + na > PPT * NT) {
        // too many for this shape's slots only: a larger shape redoes the cell
        if (can_defer && ls + na <= I.max_ppc) return -1;
        *errbits |= ERR_CAPACITY;
        const int room_log = I.max_ppc - ls, room_phys = PPT * NT - a;
        na = room_log < room_phys ? room_log : room_phys;
        if (na < 0) na = 0;
    }
    double cw = I.r_p * f.nu * pne * I.dt / 2.0;
    if (I.weight_mode == 0) cw /= m1;
    const double factor = batch == 7 ? -2.0 * (-expm1(-f.x)) / f.x : 1.0;
    const double sq = sqrt(f.theta);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int j = k * NT + tid;
        if (k * NT + NT > a && k * NT < a + na && j >= a && j < a + na) {
            const int q = j - a;
            uint32_t rr[4];
            draw(I, step, PUR_SPAWN_POS, (uint32_t)batch, (uint32_t)cell, (uint32_t)q, rr);
            const double uy = uni_d(rr[0], I.prec), ux = uni_d(rr[1], I.prec);
            P.y[k] = (real)(I.y0 + ((double)iy + uy) * I.dy);
            if (DIM == 2) P.x[k] = (real)(I.x0 + ((double)ix + ux) * I.dx);
            draw(I, step, PUR_SPAWN_VEL, (uint32_t)batch, (uint32_t)cell, (uint32_t)q, rr);
            double z[3], C[3];
            normal3_d(rr, I.prec, z);
            C[0] = sq * z[0];
            C[1] = sq * z[1];
            C[2] = sq * z[2];
            P.c0[k] = (real)(f.U[0] + C[0]);
            P.c1[k] = (real)(f.U[1] + C[1]);
            P.c2[k] = (real)(f.U[2] + C[2]);
            P.w[k] = (real)(-cw * grad_bracket(I.Pr, f, C) * factor);
            P.st[k] = (uint32_t)FT_KEEP | ((uint32_t)(ls + q) << 8);
        }
    }
    constexpr int PSB = lds_dims(NT).psb;
    if (I.proj && na >= 5) {
        // Gram matrix and right-hand side summed in batch order (the order
        // the batch was drawn in), independent of where the batch sits in
        // the registers: each batch particle leaves (psi, w) in LDS, chunk
        // by chunk, and lane e of wave 0 accumulates entry e serially.
        int er = 0, es = 0;
        if (tid < 15) {
            while ((er + 1) * (er + 2) / 2 <= tid) ++er;
            es = tid - er * (er + 1) / 2;
        }
        double acc = 0.0;
        bool mine = false;
        for (int q0 = 0; q0 < na; q0 += PSB) {
            wg_sync<NT>();
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int j = k * NT + tid;
                if (k * NT + NT > a && k * NT < a + na && j >= a + q0 && j < a + na &&
                    j < a + q0 + PSB) {
                    mine = true;
                    double psi[5];
                    psi5((double)P.c0[k], (double)P.c1[k], (double)P.c2[k], f.U, sq, f.theta,
                         psi);
                    double* ps = L.psb + 6 * (j - a - q0);
#pragma unroll
                    for (int r1 = 0; r1 < 5; ++r1) ps[r1] = psi[r1];
                    ps[5] = (double)P.w[k];
                }
            }
            wg_sync<NT>();
            if (tid < 20) {
                // one running sum in batch order, chunk after chunk (the
                // plain sum's order): an ill-conditioned Gram system (a batch
                // of a few particles) then gives the weights of the plain
                // sum, not weights off by its rounding times the condition
                // number
                const int nq = na - q0 < PSB ? na - q0 : PSB;
                const int ea = tid < 15 ? er : 5, eb = tid < 15 ? es : tid - 15;
                for (int q = 0; q < nq; ++q) acc += L.psb[6 * q + ea] * L.psb[6 * q + eb];
            }
        }
        wg_sync<NT>();
        if (tid < 20) L.sc[tid] = acc;
        wg_sync<NT>();
        // only the waves holding the batch solve and update
        if (__ballot(mine) == 0) return na;
        double g[20];
#pragma unroll
        for (int q = 0; q < 20; ++q) g[q] = L.sc[q];
        // 5x5 Gram solve, unrolled in registers (the same values in every
        // lane): Cholesky G = L L^T, then L y = b and L^T lam = y
        double Lm[5][5];
        {
            int q = 0;
#pragma unroll
            for (int r1 = 0; r1 < 5; ++r1)
#pragma unroll
                for (int s1 = 0; s1 <= r1; ++s1) Lm[r1][s1] = g[q++];
        }
        const double g00 = Lm[0][0];
        bool ok = true;
#pragma unroll
        for (int i = 0; i < 5; ++i)
#pragma unroll
            for (int jj = 0; jj <= i; ++jj) {
                double t = Lm[i][jj];
#pragma unroll
                for (int k2 = 0; k2 < jj; ++k2) t -= Lm[i][k2] * Lm[jj][k2];
                if (i == jj) {
                    ok = ok && (t > 1e-10 * g00);
                    Lm[i][i] = sqrt(t > 0.0 ? t : 1.0);
                } else {
                    Lm[i][jj] = t / Lm[jj][jj];
                }
            }
        double lam[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            double t = g[15 + i];
#pragma unroll
            for (int k2 = 0; k2 < i; ++k2) t -= Lm[i][k2] * lam[k2];
            lam[i] = t / Lm[i][i];
        }
#pragma unroll
        for (int i = 4; i >= 0; --i) {
            double t = lam[i];
#pragma unroll
            for (int k2 = i + 1; k2 < 5; ++k2) t -= Lm[k2][i] * lam[k2];
            lam[i] = t / Lm[i][i];
        }
        if (ok) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int j = k * NT + tid;
                if (k * NT + NT > a && k * NT < a + na && j >= a && j < a + na) {
                    double psi[5];
                    psi5((double)P.c0[k], (double)P.c1[k], (double)P.c2[k], f.U, sq, f.theta,
                         psi);
                    double d = 0.0;
#pragma unroll
                    for (int r1 = 0; r1 < 5; ++r1) d += psi[r1] * lam[r1];
                    P.w[k] = (real)((double)P.w[k] - d);
                }
            }
        }
    }
    return na;
}

// ---------------------------------------------------------------------------
// f_G(t) velocity of one reassigned particle (Table 2 step 6; Eq. 6c, 29-32).
// The time-sample uniform is word 2 (rt) of the particle's selection draw.
// ---------------------------------------------------------------------------
// Cholesky factor of lambda = theta (I + (1 - 1/Pr) alpha sigma/p) (Eq. 6c
// with the stress of Eq. 32), FP64; a pivot <= 1e-12 theta falls back to
// theta I (fb = 1)
struct EsFactor {
    double L00, L10, L20, L11, L21, L22;
    int fb;
};

__device__ __forceinline__ EsFactor es_factor(const InstDev& I, const CellF& f, double alpha)
{
    const double cc = (1.0 - 1.0 / I.Pr) * alpha;
    const double th = f.theta;
    const double l00 = th * (1.0 + cc * f.s[0]), l11 = th * (1.0 + cc * f.s[1]);
    const double l22 = th * (1.0 + cc * f.s[2]);
    const double l10 = th * cc * f.s[3], l20 = th * cc * f.s[4], l21 = th * cc * f.s[5];
    const double tiny = 1e-12 * th;
    EsFactor L;
    L.L00 = L.L10 = L.L20 = L.L11 = L.L21 = L.L22 = 0.0;
    L.fb = 0;
    if (!(l00 > tiny)) L.fb = 1;
    if (!L.fb) {
        L.L00 = sqrt(l00);
        const double iL00 = 1.0 / L.L00;
        L.L10 = l10 * iL00;
        L.L20 = l20 * iL00;
        const double d1 = l11 - L.L10 * L.L10;
        if (!(d1 > tiny)) L.fb = 1;
        if (!L.fb) {
            L.L11 = sqrt(d1);
            L.L21 = (l21 - L.L20 * L.L10) / L.L11;
            const double d2 = l22 - L.L20 * L.L20 - L.L21 * L.L21;
            if (!(d2 > tiny)) L.fb = 1;
            else L.L22 = sqrt(d2);
        }
    }
    if (L.fb) {
        L.L00 = L.L11 = L.L22 = sqrt(th);
        L.L10 = L.L20 = L.L21 = 0.0;
    }
    return L;
}

// the velocity u + L z of one reassigned particle (Box-Muller z of its
// RESAMPLE draw; single precision for FP32 state)
template <typename real>
__device__ __forceinline__ void es_draw(const InstDev& I, int cell, int slot, uint32_t step,
                                        const CellF& f, const EsFactor& L, real& c0, real& c1,
                                        real& c2)
{
    uint32_t r[4];
    draw(I, step, PUR_RESAMPLE, 0u, (uint32_t)cell, (uint32_t)slot, r);
    double z[3];
    if (sizeof(real) == 4) {
        float zf[3];
        normal3_f(r, zf);
        z[0] = zf[0];
        z[1] = zf[1];
        z[2] = zf[2];
    } else {
        normal3_d(r, I.prec, z);
    }
    c0 = (real)(f.U[0] + L.L00 * z[0]);
    c1 = (real)(f.U[1] + L.L10 * z[0] + L.L11 * z[1]);
    c2 = (real)(f.U[2] + L.L20 * z[0] + L.L21 * z[1] + L.L22 * z[2]);
}

// the linear map of Eq. 10-11: u + sqrt(theta) S z with S = I - (1 - Pr) /
// (2 Pr) a sigma / p; a = 1 is SP-ESBGK's target, a = alpha of Eq. 32 maps to
// f_G(t) (its covariance to first order in sigma / p).  z is the particle's
// RESAMPLE draw, in single precision for FP32 state.
template <typename real>
__device__ __forceinline__ void lin_draw(const InstDev& I, int cell, int slot, uint32_t step,
                                         const CellF& f, double a, real& c0, real& c1, real& c2)
{
    const double kk = (1.0 - I.Pr) / (2.0 * I.Pr) * a;
    const double S00 = 1.0 - kk * f.s[0], S11 = 1.0 - kk * f.s[1], S22 = 1.0 - kk * f.s[2];
    const double S01 = -kk * f.s[3], S02 = -kk * f.s[4], S12 = -kk * f.s[5];
    uint32_t r[4];
    draw(I, step, PUR_RESAMPLE, 0u, (uint32_t)cell, (uint32_t)slot, r);
    double z[3];
    if (sizeof(real) == 4) {
        float zf[3];
        normal3_f(r, zf);
        z[0] = zf[0];
        z[1] = zf[1];
        z[2] = zf[2];
    } else {
        normal3_d(r, I.prec, z);
    }
    const double sq = sqrt(f.theta);
    c0 = (real)(f.U[0] + sq * (S00 * z[0] + S01 * z[1] + S02 * z[2]));
    c1 = (real)(f.U[1] + sq * (S01 * z[0] + S11 * z[1] + S12 * z[2]));
    c2 = (real)(f.U[2] + sq * (S02 * z[0] + S12 * z[1] + S22 * z[2]));
}

// the expectation of alpha(t) (Eq. 32) over the Eq. 29-30 time distribution
// (density nu_ES e^{nu_ES t} / (e^{nu_ES dt} - 1) on [0, dt])
__device__ __forceinline__ double alpha_mean(const InstDev& I, const CellF& f, double pne)
{
    const double Pr = I.Pr, y = f.nu * I.dt;
    const double m = Pr / (Pr - 1.0) * expm1((Pr - 1.0) * y) / expm1(Pr * y);
    return pne + (1.0 - pne) * m;
}

template <typename real>
__device__ __forceinline__ int resample_one(const InstDev& I, int cell, int slot, uint32_t step,
                                            const CellF& f, double pne, uint32_t rt, real& c0,
                                            real& c1, real& c2)
{
    if (I.scheme == 1) {
        lin_draw<real>(I, cell, slot, step, f, 1.0, c0, c1, c2);
        return 0;
    }
    uint32_t r[4];
    r[2] = rt;
    double alpha;
    if (sizeof(real) == 4) {
        const float u = uni_f(r[2]);
        const float x = (float)f.x, nues = (float)(I.Pr * f.nu);
        const float tf = (float)I.dt + logf(u + (1.0f - u) * expf(-x)) / nues;
        alpha = (double)((float)pne + (1.0f - (float)pne) * expf(-(float)f.nu * tf));
    } else {
        const double u = uni_d(r[2], I.prec);
        const double t = I.dt + log(u + (1.0 - u) * exp(-f.x)) / (I.Pr * f.nu);
        alpha = pne + (1.0 - pne) * exp(-f.nu * t);
    }
    if (I.es_sampler == 1) {
        lin_draw<real>(I, cell, slot, step, f, alpha, c0, c1, c2);
        return 0;
    }
    const EsFactor L = es_factor(I, f, alpha);
    es_draw<real>(I, cell, slot, step, f, L, c0, c1, c2);
    return L.fb;
}

// k-th smallest (1-based) rank key among the selected particles.  The keys
// are 21 random bits over the 11-bit slot, so a histogram of the top bits
// (11 bits for 256-thread cells, 6 for one-wave cells of at most 512
// particles) leaves a few keys in the bucket that holds the k-th; those are
// collected (into the gather map, free during the relaxation) and ranked
// exactly by wave 0.  Keys are distinct (they end in the slot).
template <int NT, typename real, int DIM, int PPT>
__device__ __forceinline__ uint32_t kth_key_r(const Parts<real, DIM, PPT>& P, const Lds& L, int kth,
                                              int nuse, int tid)
{
    constexpr int NB = lds_dims(NT).kth;
    constexpr int SH = NB == 64 ? 26 : 21;  // bucket = the key's top log2(NB) bits
    static_assert((1 << (32 - SH)) == NB, "bucket bits");
    for (int b = tid; b < NB; b += NT) L.hist[b] = 0u;
    if (tid == 0) L.fcount[1] = 0u;
    wg_sync<NT>();
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (k * NT < nuse && fate(P, k) == FT_SEL) atomicAdd(&L.hist[P.key[k] >> SH], 1u);
    wg_sync<NT>();
    if (tid < 64) {
        // lane l owns buckets [32 l, 32 l + 32)
        uint32_t s = 0;
#pragma unroll 8
        for (int q = 0; q < NB / 64; ++q) s += L.hist[tid * (NB / 64) + q];
        uint32_t incl = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, 64);
            if (tid >= o) incl += t;
        }
        const uint32_t excl = incl - s;
        const bool here = excl < (uint32_t)kth && incl >= (uint32_t)kth;
        if (here) {
            uint32_t run = excl;
            int q = 0;
            for (; q < NB / 64; ++q) {
                const uint32_t h = L.hist[tid * (NB / 64) + q];
                if (run + h >= (uint32_t)kth) break;
                run += h;
            }
            L.wtot[62] = (uint32_t)(tid * (NB / 64) + q);  // bucket of the k-th
            L.wtot[63] = run;                              // keys below that bucket
        }
    }
    wg_sync<NT>();
    const uint32_t bucket = L.wtot[62];
    const int rem = kth - (int)L.wtot[63];
    uint32_t* cand = L.srcmap;
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (k * NT < nuse && fate(P, k) == FT_SEL && (P.key[k] >> SH) == bucket)
            cand[atomicAdd(&L.fcount[1], 1u)] = P.key[k];
    wg_sync<NT>();
    if (tid < 64) {
        const int m = (int)L.fcount[1];
        for (int i = tid; i < m; i += 64) {
            const uint32_t ki = cand[i];
            int r = 0;
            for (int j = 0; j < m; ++j) r += cand[j] < ki ? 1 : 0;
            if (r == rem - 1) L.wtot[61] = ki;
        }
    }
    wg_sync<NT>();
    return L.wtot[61];
}

// Cell scalars, computed by wave 0: lane 0 derives f from the centred
// moments m0 of n particles while lane 1 derives from the centred form of the
// averaged raw sums A (the same code on two lanes at once).  With use_avg, s
// and h of the result come from the averages (zero when those are
// degenerate).  Every lane of wave 0 returns the same values.
__device__ __forceinline__ CellF pair_derive(const InstDev& I, const double (&m0)[NMOM], int n,
                                             const double (&A)[NMOM], bool use_avg, int lane)
{
    double m[NMOM];
    if (lane == 1 && use_avg) {
        centred_from_raw(A, m);
    } else {
#pragma unroll
        for (int q = 0; q < NMOM; ++q) m[q] = m0[q];
    }
    CellF fl;
    derive(I, m, lane == 1 ? 2 : n, fl);
    CellF f;
    f.valid = __builtin_amdgcn_readlane(fl.valid, 0);
    f.S0 = readlane_d(fl.S0, 0);
#pragma unroll
    for (int q = 0; q < 3; ++q) f.U[q] = readlane_d(fl.U[q], 0);
    f.trK = readlane_d(fl.trK, 0);
    f.theta = readlane_d(fl.theta, 0);
    f.rho = readlane_d(fl.rho, 0);
    f.p = readlane_d(fl.p, 0);
    f.T = readlane_d(fl.T, 0);
    f.mu = readlane_d(fl.mu, 0);
    f.nu = readlane_d(fl.nu, 0);
    f.x = readlane_d(fl.x, 0);
    const bool avg = use_avg && f.valid;
    const int va = __builtin_amdgcn_readlane(fl.valid, 1);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double s0 = readlane_d(fl.s[q], 0), s1 = readlane_d(fl.s[q], 1);
        f.s[q] = avg ? (va ? s1 : 0.0) : s0;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double h0 = readlane_d(fl.h[q], 0), h1 = readlane_d(fl.h[q], 1);
        f.h[q] = avg ? (va ? h1 : 0.0) : h0;
    }
    return f;
}

// the shape-independent part of the gather (bin runs, far arrivals, count),
// kept when a cell is retried with more particle slots per thread
struct GatherState {
    bool ready;
    int n0, nwin, nfc;
    uint32_t err;
};

// One cell with PPT slots per thread.  Returns 0 when the cell is done (or
// the instance has failed) and 1 or 2 when it needs more slots than this
// shape has; then nothing of the cell has been written: with retry_local the
// caller reruns it with a larger shape (the gather state is reused), else
// the cell is appended to tier_out for the next launch.  carve_cap is the
// slot count the LDS tables are laid out for (the largest shape of the launch).
template <int NT, typename real, int DIM, int PPT, bool XB>
__device__ __forceinline__ int process_cell_r(const InstDev& I, int c, int mode,
                                              unsigned char* smem, int tid, int g, int* tier_out,
                                              int tier_len, int carve_cap, bool retry_local,
                                              GatherState& gs)
{
    const int* ctl = I.ctl;
    if (ctl[CTL_ERR] != 0) return 0;
    const int cur = ctl[CTL_CUR];
    const uint32_t step = (uint32_t)ctl[CTL_STEP];
    const int nsamp = ctl[CTL_NSAMP];
    const int nb = I.nb;
    constexpr int CAP = PPT * NT;
    constexpr int FAR_LDS = lds_dims(NT).far;
    const Lds L = carve<NT>(smem, carve_cap, nb);
    const int ix = c % I.nx, iy = c / I.nx;
    const bool per_x = I.face_kind[0] == 2, per_y = I.face_kind[2] == 2;
    uint32_t errbits = 0;
    double* dg = I.diag ? I.diag + (size_t)c * NDIAG : nullptr;
    // hand the cell to a larger shape (nothing of it written yet)
    const bool can_defer = retry_local || tier_out != nullptr;
    auto defer = [&](int code) -> int {
        if (!retry_local && tid == 0) {
            if (!tier_out) {
                // the last shape has nowhere to hand the cell: poison the instance
                atomicOr(&I.ctl[CTL_ERR], (int)ERR_CAPACITY);
            } else {
                const int k = atomicAdd(&tier_out[0], 1);
                if (k < tier_len) tier_out[1 + k] = g;
                else atomicOr(&I.ctl[CTL_ERR], (int)ERR_CAPACITY);  // lists not cleared
            }
        }
        return code;
    };
    // phase time stamps go to LDS (no stall on a global read-modify-write in
    // the timed code); the durations are added to the record at the end
    if (dg && tid == 0) {
        for (int k = 0; k < 15; ++k) L.tst[k] = 0;
        L.tst[15] = clock64();
    }
    auto mark = [&](int k) {
        if (dg && tid == 0) L.tst[k] = clock64();
    };
    Parts<real, DIM, PPT> P;

    if (!gs.ready) {
    // ---- gather: window bins of the neighbours, then far arrivals.  All
    // global loads of this part are issued before any of them is waited for:
    // the per-cell inputs of the lane-0 sections, the far-list length and the
    // neighbours' bin offsets (nb <= 256 bins: one per thread of a 256-thread
    // cell, a few per lane of a one-wave cell).
    double pv = 0.0;
    if (tid < 41) {
        if (tid < 13) {
            if (I.jmom_mode == 1) pv = I.avgs[(size_t)tid * I.ncell + c];
        } else if (tid < 26) {
            pv = I.avg[(size_t)(tid - 13) * I.ncell + c];
        } else if (tid < 39) {
            pv = I.mom[(size_t)(tid - 26) * I.ncell + c];
        } else {
            pv = tid == 39 ? I.pcur[c] : I.pprev[c];
        }
    }
    const int nfar_all = I.far_n[cur];
    {
        const uint32_t* tin = I.tab[cur];
        constexpr int BPT = (MAX_BINS + NT - 1) / NT;  // window bins per thread
        uint32_t len[BPT], base[BPT];
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
        const int b = q * NT + tid;
        len[q] = 0;
        base[q] = 0;
        if (b < nb) {
            const int oy = b / I.nbx - I.Ky, ox = b % I.nbx - I.Kx;
            int sy = iy + oy, sx = ix + ox;
            bool ok = true;
            if (per_y) sy = wrap(sy, I.ny);
            else ok = ok && sy >= 0 && sy < I.ny;
            if (DIM == 2) {
                if (per_x) sx = wrap(sx, I.nx);
                else ok = ok && sx >= 0 && sx < I.nx;
            } else {
                sx = 0;
            }
            if (ok) {
                const int s = sy * I.nx + sx;
                const uint32_t* t = tin + (size_t)s * (nb + 1);
                const uint32_t a0 = t[b], a1 = t[b + 1];
                len[q] = a1 - a0;
                base[q] = (uint32_t)s * (uint32_t)I.cap + a0;
            }
        }
        }
        if (tid < 41) L.pre[tid] = pv;
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int b = q * NT + tid;
            if (b < nb) {
                L.run_pre[b] = len[q];
                L.run_src[b] = base[q];
            }
        }
        if (tid == 0) L.fcount[0] = 0u;
        wg_sync<NT>();
        wave0_scan(L.run_pre, nb, tid);
        if (nfar_all > 0) {
            const uint32_t* fm = I.far_meta[cur];
            for (int e = tid; e < nfar_all && e < I.far_cap; e += NT)
                if ((int)fm[3 * e] == c) {
                    const uint32_t k = atomicAdd(&L.fcount[0], 1u);
                    if (k < (uint32_t)FAR_LDS) {
                        L.fkey[k] = ((uint64_t)fm[3 * e + 1] << 32) | (uint64_t)fm[3 * e + 2];
                        L.fent[k] = (uint32_t)e;
                    }
                }
        }
        wg_sync<NT>();
    }
    int nfc = (int)L.fcount[0];
    if (nfc > FAR_LDS) {
        errbits |= ERR_WINDOW;
        nfc = FAR_LDS;
    }
    if (nfc > 0) {
        for (int k = tid; k < nfc; k += NT) {
            const uint64_t key = L.fkey[k];
            uint32_t r = 0;
            for (int j = 0; j < nfc; ++j) r += L.fkey[j] < key ? 1u : 0u;
            const int oy = (int)((key >> 48) & 0xFFFF) - 32768;
            const int ox = (int)((key >> 32) & 0xFFFF) - 32768;
            int ib;
            if (oy < -I.Ky) ib = 0;
            else if (oy > I.Ky) ib = nb;
            else if (ox < -I.Kx) ib = (oy + I.Ky) * I.nbx;
            else ib = (oy + I.Ky + 1) * I.nbx;
            L.fpos[k] = L.run_pre[ib] + r;
            L.fib[k] = (uint32_t)ib;
        }
        wg_sync<NT>();
    }
    for (int b = tid; b < nb; b += NT) {
        uint32_t sh = 0;
        for (int k = 0; k < nfc; ++k) sh += (int)L.fib[k] <= b ? 1u : 0u;
        L.run_dst[b] = L.run_pre[b] + sh;
    }
    wg_sync<NT>();
    gs.nwin = (int)L.run_pre[nb];
    gs.nfc = nfc;
    gs.n0 = gs.nwin + nfc;
    gs.err = errbits;
    gs.ready = true;
    }
    const int nfc = gs.nfc;
    int n0 = gs.n0;
    errbits |= gs.err;
    if (can_defer && n0 <= I.max_ppc) {
        // an early hand-on, before any work on the cell: the batches this
        // pass will add, about S0 / r_p each (S0 of the cell's previous
        // moments standing in for the current one).  A pass that relaxes
        // budgets three batches (steps 4, 7 and the next step 2) whether or
        // not it also moves.  The exact tests come later (steps 4 and 7 as
        // their batches are drawn; step 2 and the entering particles of the
        // next move in every relaxing pass, the fused one as it draws them
        // and the one that only relaxes at its end), so which shape relaxes
        // a cell does not depend on how a run is split into calls (wave and
        // workgroup shapes add in different orders).  The margin weighs a
        // late hand-on, which wastes the relaxation done so far, against an
        // early one: in a one-wave cell the first is cheap and the second
        // sends the cell to a four-wave shape (S0 / r_p + 1 per batch: on
        // the slit 13 % faster than with 1.1 S0 / r_p + 8); in a workgroup
        // cell a late hand-on wastes a workgroup's relaxation
        // (1.05 S0 / r_p + 3).  A pass that only takes moments adds nothing
        // and reads no previous moments (after a state is created or loaded
        // there are none).
        const int nbat = (mode & MODE_RELAX) ? 3 : ((mode & MODE_MOVE) ? 1 : 0);
        const double sp = nbat > 0 ? fmax(L.pre[26], 0.0) : 0.0;
        const double per = NT == 64 ? sp / I.r_p + 1.0 : 1.05 * sp / I.r_p + 3.0;
        const double est = n0 + nbat * per;
        if (n0 > CAP || est > (double)CAP) return defer(1);
    }
    if (n0 > I.max_ppc || n0 > CAP) {
        errbits |= ERR_CAPACITY;
        n0 = I.max_ppc < CAP ? I.max_ppc : CAP;
    }
    // gather map: each run (one bin of one neighbour) written by a group of
    // 4 threads, interleaved over the run's particles
    for (int t = tid; t < 4 * nb; t += NT) {
        const int b = t >> 2;
        const uint32_t len = L.run_pre[b + 1] - L.run_pre[b];
        const uint32_t dst0 = L.run_dst[b], src0 = L.run_src[b];
        for (uint32_t off = (uint32_t)(t & 3); off < len; off += 4) {
            const uint32_t dst = dst0 + off;
            if ((int)dst < n0) L.srcmap[dst] = src0 + off;
        }
    }
    for (int k = tid; k < nfc; k += NT)
        if ((int)L.fpos[k] < n0) L.srcmap[L.fpos[k]] = FARBIT | L.fent[k];
    wg_sync<NT>();
    {
        const real* in[6];
        const real* fin[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            in[q] = (const real*)I.pc[cur][q];
            fin[q] = (const real*)I.far_pc[cur][q];
        }
        const int n0u = uni(n0);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int j = k * NT + tid;
            if (k * NT < n0u && j < n0) {
                const uint32_t s = L.srcmap[j];
                const real* const* src = (s & FARBIT) ? fin : in;
                const size_t e = (size_t)(s & ~FARBIT);
                if (DIM == 2) P.x[k] = src[0][e];
                P.y[k] = src[1][e];
                P.c0[k] = src[2][e];
                P.c1[k] = src[3][e];
                P.c2[k] = src[4][e];
                P.w[k] = src[5][e];
                P.st[k] = (uint32_t)FT_KEEP | ((uint32_t)j << 8);
                if (I.diag && (mode & MODE_RELAX)) {
                    // where this particle of f-tilde^* came from (the sort's record)
                    uint32_t scell, sslot;
                    if (s & FARBIT) {
                        const uint32_t* fm = I.far_meta[cur] + 3 * e;
                        int sy = iy + ((int)(fm[1] >> 16) - 32768);
                        int sx = ix + ((int)(fm[1] & 0xFFFFu) - 32768);
                        if (per_y) sy = wrap(sy, I.ny);
                        if (DIM == 2 && per_x) sx = wrap(sx, I.nx);
                        scell = (uint32_t)(sy * I.nx + (DIM == 2 ? sx : 0));
                        sslot = fm[2];
                    } else {
                        scell = (uint32_t)(e / (size_t)I.cap);
                        sslot = I.ori[cur][e];
                    }
                    I.sorg[(size_t)c * I.cap + j] = ((uint64_t)scell << 32) | sslot;
                }
            } else {
                P.st[k] = FT_EMPTY;
            }
        }
    }
    mark(0);

    int nphys = n0;  // physical positions in use
    int nlog = n0;   // live particles (logical count)
    // the workgroup-uniform cell scalars live in LDS: computed by lane 0 of
    // wave 0, read by everyone (keeps them out of the per-lane registers)
    CellF& f = *L.f;
    double* Ms = L.mom;

    if (mode & MODE_RELAX) {
        if (dg && tid == 0) {
            for (int k = 0; k < NDIAG_STEP; ++k)
                if (k != D_N2 && k != D_CLAMP && k != D_MARG_CNT2 && k != D_NINJ &&
                    k != D_NGONE && k != D_NPRE)
                    dg[k] = 0.0;
            dg[D_NIN] = n0;
        }
        {
            double cen[NMOM], rawt[NMOM], E0;
            moments_r<NT>(P, L, tid, uni(n0), cen, rawt, &E0);
            if (tid < 64) {
                const bool use_avg = I.jmom_mode == 1 && (int)step >= I.avg_start;
                double A[NMOM];
                const double ne = avg_window(I.n_avg, nsamp, I.avg_init);
#pragma unroll
                for (int q = 0; q < NMOM; ++q)
                    A[q] = (ne - 1.0) / ne * L.pre[q] + 1.0 / ne * rawt[q];
                CellF fw = pair_derive(I, cen, n0, A, use_avg, tid);
                if (fw.valid) {
                    // Eq. 33 divisors with P_ne^n
                    const double Pn = L.pre[39];
                    const double da = 1.0 + I.dt * fw.nu * Pn / 2.0;
                    const double db = 1.0 + I.dt * fw.nu * I.Pr * Pn / 2.0;
#pragma unroll
                    for (int q = 0; q < 6; ++q) fw.s[q] /= da;
#pragma unroll
                    for (int q = 0; q < 3; ++q) fw.h[q] /= db;
                }
                if (tid == 0) {
                    for (int q = 0; q < NMOM; ++q) Ms[q] = cen[q];
                    Ms[26] = E0;
                    for (int q = 0; q < 3; ++q) Ms[27 + q] = rawt[1 + q];
                    if (use_avg)
                        for (int q = 0; q < NMOM; ++q) L.pend[13 + q] = A[q];
                    f = fw;
                }
            }
            wg_sync<NT>();
        }
        mark(1);
        int flags = 0;
        if (dg && tid == 0) {
            dg[D_M0] = Ms[0];
            dg[D_P0X] = Ms[27];
            dg[D_P0Y] = Ms[28];
            dg[D_P0Z] = Ms[29];
            dg[D_E0] = Ms[26];
            dg[D_MARG_SEL] = dg[D_MARG_ROUND] = dg[D_MARG_CNT] = __builtin_inf();
        }
        if (!f.valid) {
            flags |= F_SKIP;
        } else {
            const double Pn = L.pre[39];
            double mcnt = __builtin_inf();
            // step 4
            const int n4 = spawn_r<NT>(I, P, L, 4, c, ix, iy, step, f, Pn, n0, n0, tid, &errbits,
                                   &mcnt, can_defer);
            if (n4 < 0) return defer(2);
            const int nl = n0 + n4;
            mark(2);
            // step 5
            const bool sp = I.scheme == 1;
            // Eq. 9's count as printed: the N_s smallest rank keys are selected
            const bool cnt = !sp && I.select_mode == 1;
            const double psel = -expm1(-f.x);
            double ss[2] = {0.0, 0.0};
            double msel = __builtin_inf();
            uint32_t rtime[PPT];  // word 2 of the selection draw: the f_G(t) time sample
            const int nlu = uni(nl);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int j = k * NT + tid;
                if (k * NT < nlu && j < nl) {
                    uint32_t r[4];
                    draw(I, step, PUR_SELECT, 0u, (uint32_t)c, (uint32_t)j, r);
                    const double u = uni_d(r[0], I.prec);
                    // SP-ESBGK: every particle is a candidate (Eq. 9 counts them)
                    const bool sel = sp || cnt || u < psel;
                    if (!sp && !cnt) msel = fmin(msel, fabs(u - psel));
                    P.key[k] = (r[1] & 0xFFFFF800u) | (uint32_t)j;
                    rtime[k] = r[2];
                    if (sel) {
                        P.st[k] = (P.st[k] & ~0xFFu) | FT_SEL;
                        if (!cnt) {
                            ss[0] += (double)P.w[k];
                            ss[1] += 1.0;
                        }
                    }
                }
            }
            if (cnt) {
                // N_s = nearest(N_c (1 - exp(-nu_ES dt))); the others go back
                const double v = (double)nl * psel;
                int nsel = (int)floor(v + 0.5);
                nsel = nsel < 0 ? 0 : (nsel > nl ? nl : nsel);
                msel = fabs(v - (floor(v) + 0.5));
                uint32_t ths = 0;
                if (nsel > 0 && nsel < nl) ths = kth_key_r<NT>(P, L, nsel, nlu, tid);
#pragma unroll
                for (int k = 0; k < PPT; ++k)
                    if (k * NT < nlu && fate(P, k) == FT_SEL) {
                        if (nsel == 0 || (nsel < nl && P.key[k] > ths)) {
                            P.st[k] = (P.st[k] & ~0xFFu) | FT_KEEP;
                        } else {
                            ss[0] += (double)P.w[k];
                            ss[1] += 1.0;
                        }
                    }
            }
            bsum<NT>(ss, L.red, tid);
            if (dg) msel = bmin<NT>(msel, L.red, tid);
            const int ns = (int)ss[1];
            // Eq. 28; for SP-ESBGK Eq. 9: N_c (1 - exp(-nu_ES dt))
            const double S = sp ? (double)ns * psel : ss[0];
            int nusp = (int)floor(S + 0.5);
            if (nusp < 0) nusp = 0;
            if (nusp > ns) nusp = ns;
            mark(3);
            uint32_t thr = 0;
            if (nusp > 0 && nusp < ns) thr = kth_key_r<NT>(P, L, nusp, nlu, tid);
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (k * NT < nlu && fate(P, k) == FT_SEL)
                    P.st[k] = (P.st[k] & ~0xFFu) |
                              ((nusp == ns || (nusp > 0 && P.key[k] <= thr))
                                   ? FT_REASSIGN
                                   : (sp ? FT_KEEP : FT_DELETE));
            mark(4);
            // step 6
            double fbs[1] = {0.0};
            if (I.es_mode == 1 && !sp) {
                // one Gaussian for the cell: alpha's expectation, one factor
                const double am = alpha_mean(I, f, Pn);
                if (I.es_sampler == 1) {
#pragma unroll
                    for (int k = 0; k < PPT; ++k)
                        if (k * NT < nlu && fate(P, k) == FT_REASSIGN) {
                            lin_draw<real>(I, c, k * NT + tid, step, f, am, P.c0[k], P.c1[k],
                                           P.c2[k]);
                            P.w[k] = (real)1.0;
                        }
                } else {
                    const EsFactor Lc = es_factor(I, f, am);
#pragma unroll
                    for (int k = 0; k < PPT; ++k)
                        if (k * NT < nlu && fate(P, k) == FT_REASSIGN) {
                            es_draw<real>(I, c, k * NT + tid, step, f, Lc, P.c0[k], P.c1[k],
                                          P.c2[k]);
                            fbs[0] += (double)Lc.fb;
                            P.w[k] = (real)1.0;
                        }
                }
            } else {
#pragma unroll
                for (int k = 0; k < PPT; ++k)
                    if (k * NT < nlu && fate(P, k) == FT_REASSIGN) {
                        fbs[0] += (double)resample_one(I, c, k * NT + tid, step, f, Pn, rtime[k],
                                                       P.c0[k], P.c1[k], P.c2[k]);
                        P.w[k] = (real)1.0;
                    }
            }
            mark(5);
            // step 7
            const int n7 = spawn_r<NT>(I, P, L, 7, c, ix, iy, step, f, Pn, nl, nl, tid, &errbits,
                                   &mcnt, can_defer);
            if (n7 < 0) return defer(2);
            nphys = nl + n7;
            mark(6);
            // conservation of the cell's mass, momentum and energy
            double WrOut = 0.0, s2Out = 0.0;
            if (I.conserve_mode == 0) {
                double cs[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) cs[q] = 0.0;
                const int npu = uni(nphys);
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    if (k * NT >= npu) continue;
                    const int fk = fate(P, k);
                    const double w = (double)P.w[k];
                    const double c0 = (double)P.c0[k], c1 = (double)P.c1[k];
                    const double c2 = (double)P.c2[k];
                    if (fk == FT_KEEP) {
                        cs[0] += w;
                        cs[1] += w * c0;
                        cs[2] += w * c1;
                        cs[3] += w * c2;
                        cs[4] += 0.5 * w * (c0 * c0 + c1 * c1 + c2 * c2);
                    } else if (fk == FT_REASSIGN) {
                        cs[5] += c0;
                        cs[6] += c1;
                        cs[7] += c2;
                        cs[8] += c0 * c0 + c1 * c1 + c2 * c2;
                    }
                }
                bsum<NT>(cs, L.red, tid);
                if (nusp == 0) {
                    flags |= F_NOUSP;
                } else {
                    const double M0 = Ms[0];
                    const double Wr = (M0 - cs[0]) / nusp;
                    WrOut = Wr;
                    // a correction only where it is one: common weight in
                    // [1/2, 2], mean shift within 3 rms spreads, scale in [1/3, 3]
                    double a[3], cb[3], sc = 1.0;
                    bool shift = true;
                    if (!(Wr >= 0.5 && Wr <= 2.0)) {
                        flags |= F_FAILMASS;
                    } else {
                        const double MR = Wr * nusp;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            a[q] = (Ms[27 + q] - cs[1 + q]) / MR;
                            cb[q] = cs[5 + q] / nusp;
                        }
                        // sum over the reassigned of |c - cb|^2, from the same
                        // pass: sum |c|^2 - |sum c|^2 / N_usp (FP64)
                        const double D = cs[8] - nusp * (cb[0] * cb[0] + cb[1] * cb[1] +
                                                         cb[2] * cb[2]);
                        const double a2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
                        double da2 = 0.0;
#pragma unroll
                        for (int q = 0; q < 3; ++q) da2 += (a[q] - cb[q]) * (a[q] - cb[q]);
                        if (nusp >= 2 && D > 0.0) {
                            if (!(da2 <= 9.0 * D / nusp)) {
                                // the mean would move by more than 3 rms spreads
                                shift = false;
                                flags |= F_FAILENERGY;
                            } else {
                                const double s2 =
                                    (Ms[26] - cs[4] - 0.5 * MR * a2) / (0.5 * Wr * D);
                                s2Out = s2;
                                if (s2 >= 1.0 / 9.0 && s2 <= 9.0) sc = sqrt(s2);
                                else flags |= F_FAILENERGY;
                            }
                        } else {
                            flags |= F_FAILENERGY;
                        }
                    }
                    // where the reassigned particles alone cannot carry it:
                    // W_r on them (mass), then one shift and scale of every
                    // particle that stays in the cell (momentum, energy), with
                    // at least two reassigned, W_r > 0, a positive thermal
                    // energy K of the set, a shift within 3 rms thermal speeds
                    // and a scale^2 in [1/4, 4]
                    bool whole = false;
                    double aw[3], uw[3], sw = 1.0;
                    if (nusp >= 2 && (flags & (F_FAILMASS | F_FAILENERGY))) {
                        const double M = cs[0] + Wr * nusp;
                        double u2 = 0.0, a2 = 0.0, du2 = 0.0;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            uw[q] = (cs[1 + q] + Wr * cs[5 + q]) / M;
                            aw[q] = Ms[27 + q] / M0;
                            u2 += uw[q] * uw[q];
                            a2 += aw[q] * aw[q];
                            du2 += (aw[q] - uw[q]) * (aw[q] - uw[q]);
                        }
                        const double K = cs[4] + 0.5 * Wr * cs[8] - 0.5 * M * u2;
                        const double s2 = (Ms[26] - 0.5 * M0 * a2) / K;
                        whole = Wr > 0.0 && M > 0.0 && K > 0.0 && du2 <= 9.0 * 2.0 * K / M &&
                                s2 >= 0.25 && s2 <= 4.0;
                        if (whole) {
                            sw = sqrt(s2);
                            flags = (flags & ~(F_FAILMASS | F_FAILENERGY)) | F_WHOLE;
                        }
                    }
                    if (whole) {
#pragma unroll
                        for (int k = 0; k < PPT; ++k) {
                            if (k * NT >= npu) continue;
                            const int fk = fate(P, k);
                            if (fk != FT_KEEP && fk != FT_REASSIGN) continue;
                            if (fk == FT_REASSIGN) P.w[k] = (real)Wr;
                            P.c0[k] = (real)(aw[0] + sw * ((double)P.c0[k] - uw[0]));
                            P.c1[k] = (real)(aw[1] + sw * ((double)P.c1[k] - uw[1]));
                            P.c2[k] = (real)(aw[2] + sw * ((double)P.c2[k] - uw[2]));
                        }
                    } else if (!(flags & F_FAILMASS)) {
#pragma unroll
                        for (int k = 0; k < PPT; ++k)
                            if (k * NT < nlu && fate(P, k) == FT_REASSIGN) {
                                if (shift) {
                                    P.c0[k] = (real)(a[0] + sc * ((double)P.c0[k] - cb[0]));
                                    P.c1[k] = (real)(a[1] + sc * ((double)P.c1[k] - cb[1]));
                                    P.c2[k] = (real)(a[2] + sc * ((double)P.c2[k] - cb[2]));
                                }
                                P.w[k] = (real)Wr;
                            }
                    }
                }
            }
            double fbt[1] = {fbs[0]};
            if (dg) bsum<NT>(fbt, L.red, tid);  // diagnostics only
            mark(7);
            // logical slots of the survivors (slot order), step-7 particles last
            {
                bool alive[PPT];
                int pre[PPT];
#pragma unroll
                for (int k = 0; k < PPT; ++k) alive[k] = fate(P, k) <= FT_REASSIGN;
                nlog = phys_scan<NT>(alive, pre, L.wtot, tid);
#pragma unroll
                for (int k = 0; k < PPT; ++k)
                    if (alive[k]) P.st[k] = (P.st[k] & 0xFFu) | ((uint32_t)pre[k] << 8);
            }
            if (nl + n7 > I.max_ppc) errbits |= ERR_CAPACITY;
            mark(8);
            if (dg && tid == 0) {
                dg[D_N4] = n4;
                dg[D_PSEL] = psel;
                dg[D_MARG_SEL] = msel;
                dg[D_MARG_ROUND] = fabs(S - (floor(S) + 0.5));
                dg[D_SSEL] = S;
                dg[D_NSEL] = ns;
                dg[D_NUSP] = nusp;
                dg[D_NDEL] = sp ? 0 : ns - nusp;
                dg[D_N7] = n7;
                dg[D_CHOLFB] = fbt[0];
                dg[D_MARG_CNT] = mcnt;
                dg[D_WR] = WrOut;
                dg[D_S2] = s2Out;
            }
        }
        // step 8: moments of f^{n+1}, Eq. 34 averages
        {
            double cen1[NMOM], raw1[NMOM], E1;
            moments_r<NT>(P, L, tid, uni(nphys), cen1, raw1, &E1);
            if (tid == 0) {
                // a moment that is not a finite number poisons the instance
                bool fin = true;
                for (int q = 0; q < NMOM; ++q) fin = fin && isfinite(raw1[q]);
                if (!fin) errbits |= ERR_NONFINITE;
                L.pend[26] = (double)nlog;
                const double ne = avg_window(I.n_avg, nsamp, I.avg_init);
                for (int q = 0; q < NMOM; ++q) {
                    Ms[q] = cen1[q];
                    L.pend[q] = raw1[q];
                    const double A = L.pre[13 + q];
                    Ms[13 + q] =
                        (int)step >= I.avg_start ? (ne - 1.0) / ne * A + 1.0 / ne * raw1[q] : A;
                }
                if (dg) {
                    dg[D_FLAGS] = flags;
                    dg[D_NOUT] = nlog;
                    dg[D_M1] = raw1[0];
                    dg[D_P1X] = raw1[1];
                    dg[D_P1Y] = raw1[2];
                    dg[D_P1Z] = raw1[3];
                    dg[D_E1] = E1;
                }
            }
        }
        mark(9);
    } else if (mode & MODE_MOMENTS) {
        double cen1[NMOM], raw1[NMOM], E1;
        moments_r<NT>(P, L, tid, uni(nphys), cen1, raw1, &E1);
        if (tid == 0) {
            L.pend[26] = (double)nlog;
            for (int q = 0; q < NMOM; ++q) {
                Ms[q] = cen1[q];
                L.pend[q] = raw1[q];
                Ms[13 + q] = L.pre[13 + q];
            }
        }
    }
    // the cell's moments (and J-moment averages) go to HBM only once no
    // larger shape can take the cell over
    auto commit = [&]() {
        if (tid != 0) return;
        if (mode & (MODE_RELAX | MODE_MOMENTS)) {
            I.cnt[c] = (int)L.pend[26];
            for (int q = 0; q < NMOM; ++q) {
                I.mom[(size_t)q * I.ncell + c] = Ms[q];
                I.raw[(size_t)q * I.ncell + c] = L.pend[q];
                I.avg[(size_t)q * I.ncell + c] = Ms[13 + q];
            }
        }
        if ((mode & MODE_RELAX) && I.jmom_mode == 1 && (int)step >= I.avg_start)
            for (int q = 0; q < NMOM; ++q) I.avgs[(size_t)q * I.ncell + c] = L.pend[13 + q];
    };

    real* out[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) out[q] = (real*)I.pc[1 - cur][q];
    uint32_t* tout = I.tab[1 - cur] + (size_t)c * (nb + 1);
    const size_t rbase = (size_t)c * I.cap;

    if (mode & MODE_MOVE) {
        const uint32_t mstep = (mode & MODE_RELAX) ? step + 1 : step;
        // cell scalars of f^{n+1} (or f^n when no relaxation ran) for step 2,
        // derived by wave 0 while every wave starts step 3 on the particles
        // already present (which does not need them)
        if (tid < 64) {
            const bool have = (mode & (MODE_RELAX | MODE_MOMENTS)) != 0;
            double m[NMOM], A[NMOM];
#pragma unroll
            for (int q = 0; q < NMOM; ++q) {
                m[q] = have ? Ms[q] : L.pre[26 + q];
                A[q] = have ? Ms[13 + q] : L.pre[13 + q];
            }
            const int ns_after =
                nsamp + (((mode & MODE_RELAX) && (int)step >= I.avg_start) ? 1 : 0);
            const CellF fw = pair_derive(I, m, nlog, A,
                                         I.jmom_mode == 1 && (ns_after > 0 || I.avg_init), tid);
            if (tid == 0) f = fw;
        }
        // step 3 for particles at physical positions [lo, hi): advect, walls,
        // destination bin; a particle leaving the sort window is marked and
        // goes to the far list only once the cell can no longer be handed on
        int clamps = 0, gone = 0;
        // sort-window bin of destination cell d (FAR_PENDING: beyond the window)
        auto bin_key = [&](int d) -> uint32_t {
            const int dy_ = DIM == 2 ? d / I.nx : d;
            const int dx_ = DIM == 2 ? d - dy_ * I.nx : 0;
            const int oy = min_image(iy - dy_, I.ny, per_y);
            const int ox = DIM == 2 ? min_image(ix - dx_, I.nx, per_x) : 0;
            if (oy < -I.Ky || oy > I.Ky || ox < -I.Kx || ox > I.Kx) return FAR_PENDING;
            return (uint32_t)((oy + I.Ky) * I.nbx + (ox + I.Kx));
        };
        auto move = [&](int lo, int hi, bool reset) {
            const int hiu = uni(hi);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int j = k * NT + tid;
                if (k * NT < hiu && j >= lo && j < hi && fate(P, k) <= FT_REASSIGN) {
                    real px = DIM == 2 ? P.x[k] : (real)0;
                    real py = P.y[k];
                    real v0 = P.c0[k], v1 = P.c1[k], v2 = P.c2[k];
                    const int slot = (int)(P.st[k] >> 8);
                    const int d =
                        advect<real, DIM, XB>(I, px, py, v0, v1, v2, c, slot, mstep, &clamps);
                    if (DIM == 2) P.x[k] = px;
                    P.y[k] = py;
                    P.c0[k] = v0;
                    P.c1[k] = v1;
                    P.c2[k] = v2;
                    // a particle gone through an open face is not written
                    if (XB && d < 0) {
                        P.key[k] = FAR_BIN;
                        ++gone;
                    } else {
                        P.key[k] = bin_key(d);
                    }
                } else if (reset) {
                    P.key[k] = FAR_BIN;
                }
            }
        };
        const int nphys0 = nphys;
        move(0, nphys0, true);
        wg_sync<NT>();
        const double P2 = (mode & MODE_RELAX) ? L.pre[39] : L.pre[40];
        double mc2 = __builtin_inf();
        // step 2 of the next time level
        const int n2 = spawn_r<NT>(I, P, L, 2, c, ix, iy, mstep, f, P2, nphys, nlog, tid, &errbits,
                               &mc2, can_defer);
        if (n2 < 0) return defer(2);
        // particles entering through open faces: counted before the last
        // capacity decision, created after the step-2 particles (slots in
        // face order)
        int ninj[4] = {0, 0, 0, 0};
        int nin = 0;
        if (XB && I.open_mask) {
#pragma unroll
            for (int fc = 0; fc < 4; ++fc) {
                ninj[fc] = inject_count<DIM>(I, c, ix, iy, fc, mstep);
                nin += ninj[fc];
            }
            const int need_log = nlog + n2 + nin, need_phys = nphys + n2 + nin;
            if (need_log > I.max_ppc || need_phys > CAP) {
                if (can_defer && need_log <= I.max_ppc) return defer(2);
                errbits |= ERR_CAPACITY;
                int room = I.max_ppc - nlog - n2 < CAP - nphys - n2 ? I.max_ppc - nlog - n2
                                                                    : CAP - nphys - n2;
                room = room < 0 ? 0 : room;
                nin = 0;
#pragma unroll
                for (int fc = 0; fc < 4; ++fc) {
                    ninj[fc] = ninj[fc] < room - nin ? ninj[fc] : room - nin;
                    nin += ninj[fc];
                }
            }
        }
        commit();
        nphys += n2;
        nlog += n2;
        mark(10);
        if (n2 > 0) move(nphys0, nphys, false);
        if (XB && nin > 0) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int j = k * NT + tid;
                if (k * NT + NT > nphys && k * NT < nphys + nin && j >= nphys &&
                    j < nphys + nin) {
                    const int q = j - nphys;
                    int fq = 0, qf = q, acc = 0;
#pragma unroll
                    for (int fc = 0; fc < 4; ++fc) {
                        if (q >= acc && q < acc + ninj[fc]) {
                            fq = fc;
                            qf = q - acc;
                        }
                        acc += ninj[fc];
                    }
                    real px = (real)0, py = (real)0, v0 = (real)0, v1 = (real)0, v2 = (real)0;
                    const int d = inject_one<real, DIM>(I, c, ix, iy, fq, qf, nlog + q, mstep, px,
                                                        py, v0, v1, v2, &clamps);
                    if (DIM == 2) P.x[k] = px;
                    P.y[k] = py;
                    P.c0[k] = v0;
                    P.c1[k] = v1;
                    P.c2[k] = v2;
                    P.w[k] = (real)1;
                    P.st[k] = (uint32_t)FT_KEEP | ((uint32_t)(nlog + q) << 8);
                    P.key[k] = d < 0 ? (uint32_t)FAR_BIN : bin_key(d);
                    gone += d < 0;
                }
            }
            nphys += nin;
            nlog += nin;
        }
        // far movers: appended now, with their destination cell and offsets
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (P.key[k] == FAR_PENDING) {
                const int d = cell_index<real, DIM>(I, DIM == 2 ? P.x[k] : (real)0, P.y[k]);
                const int dy_ = DIM == 2 ? d / I.nx : d;
                const int dx_ = DIM == 2 ? d - dy_ * I.nx : 0;
                const int oy = min_image(iy - dy_, I.ny, per_y);
                const int ox = DIM == 2 ? min_image(ix - dx_, I.nx, per_x) : 0;
                const int slot = (int)(P.st[k] >> 8);
                const int e = atomicAdd(&I.far_n[1 - cur], 1);
                if (e < I.far_cap) {
                    uint32_t* fm = I.far_meta[1 - cur] + 3 * (size_t)e;
                    fm[0] = (uint32_t)d;
                    fm[1] = ((uint32_t)(oy + 32768) << 16) | (uint32_t)(ox + 32768);
                    fm[2] = (uint32_t)slot;
                    real* const* fo = (real* const*)I.far_pc[1 - cur];
                    if (DIM == 2) fo[0][e] = P.x[k];
                    fo[1][e] = P.y[k];
                    fo[2][e] = P.c0[k];
                    fo[3][e] = P.c1[k];
                    fo[4][e] = P.c2[k];
                    fo[5][e] = P.w[k];
                } else {
                    errbits |= ERR_WINDOW;
                }
                P.key[k] = FAR_BIN;
            }
        }
        mark(11);
        // stable ranks by bin over physical positions (tiles of 64)
        const int ntl = (nphys + 63) / 64;
        for (int q = tid; q < ntl * nb; q += NT) L.tiles[q] = 0;
        wg_sync<NT>();
        const int lane = tid & 63;
        // lanes of a wave that share a bin, found bit by bit of the bin
        // index (one ballot per bit instead of one per distinct bin)
        const int nbits = 32 - __clz(nb - 1 > 0 ? nb - 1 : 1);
        const int npu_t = uni(nphys);
        uint32_t rank[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int j = k * NT + tid;
            const bool act = P.key[k] != (uint32_t)FAR_BIN;
            const int b = (int)P.key[k];
            const int tile = j >> 6;
            rank[k] = 0;
            if (k * NT >= npu_t) continue;
            uint64_t peers = __ballot(act);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                if (bit < nbits) {
                    const bool on = act && ((b >> bit) & 1);
                    const uint64_t m = __ballot(on);
                    peers &= ((b >> bit) & 1) ? m : ~m;
                }
            }
            if (act) {
                rank[k] = (uint32_t)__popcll(peers & lanemask_lt(lane));
                if (rank[k] == 0) L.tiles[tile * nb + b] = (uint16_t)__popcll(peers);
            }
        }
        wg_sync<NT>();
        for (int b = tid; b < nb; b += NT) {
            uint32_t s = 0;
            for (int t = 0; t < ntl; ++t) s += L.tiles[t * nb + b];
            L.boff[b] = s;
        }
        wg_sync<NT>();
        wave0_scan(L.boff, nb, tid);
        wg_sync<NT>();
        for (int b = tid; b < nb; b += NT) {
            uint32_t run = L.boff[b];
            for (int t = 0; t < ntl; ++t) {
                const uint32_t v = L.tiles[t * nb + b];
                L.tiles[t * nb + b] = (uint16_t)run;
                run += v;
            }
        }
        wg_sync<NT>();
        mark(12);
        // write-out: each particle straight from its registers
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (P.key[k] != (uint32_t)FAR_BIN) {
                const int j = k * NT + tid;
                const uint32_t pos = (uint32_t)L.tiles[(j >> 6) * nb + P.key[k]] + rank[k];
                if (DIM == 2) out[0][rbase + pos] = P.x[k];
                out[1][rbase + pos] = P.y[k];
                out[2][rbase + pos] = P.c0[k];
                out[3][rbase + pos] = P.c1[k];
                out[4][rbase + pos] = P.c2[k];
                out[5][rbase + pos] = P.w[k];
                if (I.diag) I.ori[1 - cur][rbase + pos] = P.st[k] >> 8;
            }
        }
        for (int b = tid; b <= nb; b += NT) tout[b] = L.boff[b];
        mark(13);
        if (dg) {
            double cl[2] = {(double)clamps, (double)gone};
            bsum<NT>(cl, L.red, tid);
            if (tid == 0) {
                dg[D_N2] = n2;
                dg[D_CLAMP] = cl[0];
                dg[D_MARG_CNT2] = mc2;
                dg[D_NINJ] = nin;
                dg[D_NGONE] = cl[1];
                dg[D_NPRE] = nlog;
            }
        }
    } else {
        if ((mode & MODE_RELAX) && can_defer) {
            // a relaxing pass that does not move tests the next move's
            // additions as the fused pass does (step 2 of the next time
            // level, then the entering particles): a cell that the fused
            // pass would hand on here is handed on here too
            const uint32_t mstep = step + 1;
            if (tid < 64) {
                double m[NMOM], A[NMOM];
#pragma unroll
                for (int q = 0; q < NMOM; ++q) {
                    m[q] = Ms[q];
                    A[q] = Ms[13 + q];
                }
                const int ns_after = nsamp + ((int)step >= I.avg_start ? 1 : 0);
                const CellF fw = pair_derive(I, m, nlog, A,
                                             I.jmom_mode == 1 && (ns_after > 0 || I.avg_init), tid);
                if (tid == 0) f = fw;
            }
            wg_sync<NT>();
            int n2w = spawn_count(I, 2, c, mstep, f, L.pre[39], nullptr);
            if (nlog + n2w > I.max_ppc || nphys + n2w > CAP) {
                if (nlog + n2w <= I.max_ppc) return defer(2);
                // the fused pass clamps the batch to the room left here
                n2w = I.max_ppc - nlog < CAP - nphys ? I.max_ppc - nlog : CAP - nphys;
                n2w = n2w < 0 ? 0 : n2w;
            }
            if (XB && I.open_mask) {
                int ninw = 0;
#pragma unroll
                for (int fc = 0; fc < 4; ++fc) ninw += inject_count<DIM>(I, c, ix, iy, fc, mstep);
                const int need_log = nlog + n2w + ninw, need_phys = nphys + n2w + ninw;
                if ((need_log > I.max_ppc || need_phys > CAP) && need_log <= I.max_ppc)
                    return defer(2);
            }
        }
        commit();
        // stay layout: every live particle at its logical slot of its own cell
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (fate(P, k) <= FT_REASSIGN) {
                const uint32_t pos = P.st[k] >> 8;
                if (DIM == 2) out[0][rbase + pos] = P.x[k];
                out[1][rbase + pos] = P.y[k];
                out[2][rbase + pos] = P.c0[k];
                out[3][rbase + pos] = P.c1[k];
                out[4][rbase + pos] = P.c2[k];
                out[5][rbase + pos] = P.w[k];
            }
        }
        const int centre = I.Ky * I.nbx + I.Kx;
        for (int b = tid; b <= nb; b += NT) tout[b] = b <= centre ? 0u : (uint32_t)nlog;
    }
    if (nlog > I.max_ppc || nphys > CAP) errbits |= ERR_CAPACITY;
    if (dg && tid == 0) dg[D_SHAPE_SLOTS] = (double)CAP;
    const uint64_t em = __ballot(errbits != 0);
    if (em) {
        uint32_t e = errbits;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) e |= __shfl_xor(e, o, 64);
        if ((tid & 63) == 0) atomicOr(&I.ctl[CTL_ERR], (int)e);
    }
    if (dg && tid == 0) {
        long long prev = L.tst[15];
        for (int k = 0; k < 15; ++k) {
            const long long t = L.tst[k];
            if (t != 0) {
                dg[NDIAG_STEP + k] += (double)(t - prev);
                prev = t;
            }
        }
    }
    return 0;
}

// Waves per SIMD asked of the register allocator (the second launch bound):
// the kernel waits on memory, LDS and barriers about half of its time, so
// more cells in flight pay for some register spills: 4 for the 1-, 2- and
// 4-slot workgroup shapes (128 VGPRs), 3 for 4|6 (168 VGPRs); measured 9 %
// (C2 pair) to 32 % (cavity) faster than without spills at 3 and 2
// workgroups per CU.  One-wave cells: 3 waves per SIMD with 4 slots per lane
// (168 VGPRs, 12 cells per CU) and 2 with 6 (256 VGPRs, 8 cells per CU):
// at 4 waves the 4-slot kernel spilled 400 B per lane (the slit pair 15 %
// slower) and the 6-slot kernel more (the cavity triple 20 % slower).
template <int NT, int PPT, int PPT2>
constexpr int cell_waves_per_simd()
{
    if (NT == 64) return PPT <= 4 ? 3 : 2;
    return PPT2 > 0 ? 3 : (PPT <= 4 ? 4 : 1);
}

template <typename real, int DIM, int NT, int PPT, int PPT2, bool XB>
__global__ void __launch_bounds__(NT, (cell_waves_per_simd<NT, PPT, PPT2>())) cell_kernel(Batch B)
{
    // one workgroup per cell (no loop over cells: a loop would let the
    // compiler hoist constants across the whole cell body)
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    int g = blockIdx.x;
    if (B.tier_in) {
        // cells left over by the next smaller shape
        if (g >= B.tier_in[0]) return;
        g = B.tier_in[1 + g];
    }
    if (g >= B.ncells) return;
    int lo = 0, hi = B.ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.base[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    GatherState gs;
    gs.ready = false;
    const InstDev& I = B.inst[lo];
    const int c = g - B.base[lo];
    if constexpr (PPT2 == 0) {
        process_cell_r<NT, real, DIM, PPT, XB>(I, c, B.mode, smem, tid, g, B.tier_out, B.ncells,
                                           NT * PPT, false, gs);
    } else {
        // PPT slots per thread first; cells that need more rerun with PPT2
        if (process_cell_r<NT, real, DIM, PPT, XB>(I, c, B.mode, smem, tid, g, nullptr, 0, NT * PPT2,
                                               true, gs) != 0)
            process_cell_r<NT, real, DIM, PPT2, XB>(I, c, B.mode, smem, tid, g, B.tier_out, B.ncells,
                                                NT * PPT2, false, gs);
    }
}

// XB: the extended boundary set (open faces, the internal plate); instances
// without them run the variant that leaves that code out.  The 6-slot wave
// shape exists without it only: with it the compiler makes the step-2
// added-particle routine an out-of-line call (as in the 8-slot workgroup
// shapes), and every one-wave kernel that runs is kept free of calls.
#define USP_CELL_INST(R, D, NT, PPT, PPT2, XB) \
    template __global__ void cell_kernel<R, D, NT, PPT, PPT2, XB>(Batch);
#define USP_CELL_ALL(R, D, XB)            \
    USP_CELL_INST(R, D, 256, 1, 0, XB)    \
    USP_CELL_INST(R, D, 256, 2, 0, XB)    \
    USP_CELL_INST(R, D, 256, 4, 0, XB)    \
    USP_CELL_INST(R, D, 256, 4, 6, XB)    \
    USP_CELL_INST(R, D, 256, 8, 0, XB)    \
    USP_CELL_INST(R, D, 64, 4, 0, XB)
#define USP_CELL_W6(R, D) USP_CELL_INST(R, D, 64, 6, 0, false)

}  // namespace usp
