// Device-side building blocks of the USP-ESBGK cell kernel: counter-based
// random numbers, cell scalars, workgroup reductions and scans.
#pragma once

#include "usp_common.h"

namespace usp {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds of: multiply
// words 0 and 2 by the Philox multipliers, mix the high halves with words 1, 3
// and the round key; the key advances by the two Weyl constants per round.
// Counter = (step, purpose << 24 | sub, cell, slot); key = the 64-bit seed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1, uint32_t r[4])
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // each 32 x 32 -> 64-bit product in one instruction (v_mad_u64_u32)
        // rather than separate low and high multiplies
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    r[0] = c0;
    r[1] = c1;
    r[2] = c2;
    r[3] = c3;
}

__device__ __forceinline__ void draw(const InstDev& I, uint32_t step, uint32_t purpose,
                                     uint32_t sub, uint32_t cell, uint32_t slot, uint32_t r[4])
{
    philox(step, (purpose << 24) | (sub & 0xFFFFFFu), cell, slot, I.key0, I.key1, r);
}

// uniform in (0,1): 23-bit grid for single-precision state (exact in float),
// 32-bit grid for double state
__device__ __forceinline__ double uni_d(uint32_t r, int prec)
{
    return prec == 32 ? ((double)(r >> 9) + 0.5) * 0x1p-23 : ((double)r + 0.5) * 0x1p-32;
}
__device__ __forceinline__ float uni_f(uint32_t r) { return ((float)(r >> 9) + 0.5f) * 0x1p-23f; }

// Box-Muller: z0, z1 from (u0, u1), z2 from (u2, u3); double precision
__device__ __forceinline__ void normal3_d(const uint32_t r[4], int prec, double z[3])
{
    const double u0 = uni_d(r[0], prec), u1 = uni_d(r[1], prec);
    const double u2 = uni_d(r[2], prec), u3 = uni_d(r[3], prec);
    const double a = sqrt(-2.0 * log(u0)), b = sqrt(-2.0 * log(u2));
    double s, c;
    sincospi(2.0 * u1, &s, &c);
    z[0] = a * c;
    z[1] = a * s;
    z[2] = b * cospi(2.0 * u3);
}

// the same in single precision (single-precision state, resampled particles)
__device__ __forceinline__ void normal3_f(const uint32_t r[4], float z[3])
{
    const float u0 = uni_f(r[0]), u1 = uni_f(r[1]), u2 = uni_f(r[2]), u3 = uni_f(r[3]);
    const float a = sqrtf(-2.0f * logf(u0)), b = sqrtf(-2.0f * logf(u2));
    float s, c;
    sincospif(2.0f * u1, &s, &c);
    z[0] = a * c;
    z[1] = a * s;
    z[2] = b * cospif(2.0f * u3);
}

// ---------------------------------------------------------------------------
// Cell scalars from centred moments (S0, U[3], K[6], Q[3]); Eq. 1, 4, 6, 35
// ---------------------------------------------------------------------------
struct CellF {
    int valid;
    double S0, U[3], trK, theta, rho, p, T, mu, nu, x;
    double s[6];  // sigma / p
    double h[3];  // q / p
};

__device__ __forceinline__ void derive(const InstDev& I, const double* m, int n, CellF& f)
{
    f.S0 = m[0];
    f.U[0] = m[1];
    f.U[1] = m[2];
    f.U[2] = m[3];
    f.trK = m[4] + m[5] + m[6];
    f.valid = (n >= 2) && (f.S0 > 0.0) && (f.trK > 0.0);
    f.theta = f.rho = f.p = f.T = f.mu = f.nu = f.x = 0.0;
    for (int k = 0; k < 6; ++k) f.s[k] = 0.0;
    for (int k = 0; k < 3; ++k) f.h[k] = 0.0;
    if (!f.valid) return;
    const double third = f.trK / 3.0;
    f.theta = third / f.S0;
    f.rho = I.F * f.S0;
    f.p = I.F * third;
    f.T = f.theta / I.R;
    // Eq. 35; the square root for hard spheres (omega = 1/2), a tenth of
    // the instructions of the general power
    const double tr = f.T / I.T_ref;
    f.mu = I.mu_ref * (I.omega == 0.5 ? sqrt(tr) : pow(tr, I.omega));
    f.nu = f.p / f.mu;
    f.x = I.Pr * f.nu * I.dt;
    // sigma / p and q / p: one division, then products
    const double inv = 1.0 / third;
    f.s[0] = (m[4] - third) * inv;
    f.s[1] = (m[5] - third) * inv;
    f.s[2] = (m[6] - third) * inv;
    f.s[3] = m[7] * inv;
    f.s[4] = m[8] * inv;
    f.s[5] = m[9] * inv;
    for (int k = 0; k < 3; ++k) f.h[k] = 0.5 * m[10 + k] * inv;
}

// centred moments from raw sums (S0, S1[3], S2[6], S3[3])
__device__ __forceinline__ void centred_from_raw(const double* r, double* m)
{
    const double s0 = r[0];
    double U[3] = {0.0, 0.0, 0.0};
    if (s0 != 0.0)
        for (int k = 0; k < 3; ++k) U[k] = r[1 + k] / s0;
    m[0] = s0;
    for (int k = 0; k < 3; ++k) m[1 + k] = U[k];
    m[4] = r[4] - s0 * U[0] * U[0];
    m[5] = r[5] - s0 * U[1] * U[1];
    m[6] = r[6] - s0 * U[2] * U[2];
    m[7] = r[7] - s0 * U[0] * U[1];
    m[8] = r[8] - s0 * U[0] * U[2];
    m[9] = r[9] - s0 * U[1] * U[2];
    const double trR = r[4] + r[5] + r[6];
    const double U2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    const double R2[3][3] = {{r[4], r[7], r[8]}, {r[7], r[5], r[9]}, {r[8], r[9], r[6]}};
    for (int i = 0; i < 3; ++i) {
        const double UR = U[0] * R2[0][i] + U[1] * R2[1][i] + U[2] * R2[2][i];
        m[10 + i] = r[10 + i] - U[i] * trR - 2.0 * UR + 2.0 * s0 * U2 * U[i];
    }
}

// Grad-13 bracket of Eq. 15 / 26 at peculiar velocity C
__device__ __forceinline__ double grad_bracket(double Pr, const CellF& f, const double C[3])
{
    const double* s = f.s;
    const double sCC = s[0] * C[0] * C[0] + s[1] * C[1] * C[1] + s[2] * C[2] * C[2] +
                       2.0 * (s[3] * C[0] * C[1] + s[4] * C[0] * C[2] + s[5] * C[1] * C[2]);
    const double C2 = C[0] * C[0] + C[1] * C[1] + C[2] * C[2];
    const double hC = f.h[0] * C[0] + f.h[1] * C[1] + f.h[2] * C[2];
    return sCC / (2.0 * f.theta) + 0.4 * Pr * hC * (C2 / (2.0 * f.theta) - 2.5) / f.theta;
}

// Eq. 34 window: running mean for the first n_avg samples, then exponential;
// with averages started from the exact initial moments, n_avg throughout
__device__ __forceinline__ double avg_window(int n_avg, int n_samples, int avg_init)
{
    const int k = n_samples + 1;
    if (avg_init) return (double)n_avg;
    return (double)(k < n_avg ? k : n_avg);
}

// ---------------------------------------------------------------------------
// Wavefront / workgroup reductions (deterministic: fixed butterfly order)
// ---------------------------------------------------------------------------
// one DPP lane move of a double (two 32-bit moves); lanes without a source,
// or outside ROWMASK, receive +0.0
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWMASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double x, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active): row shifts by
// 1, 2, 4, 8 leave each 16-lane row's total in its lane 15; two row
// broadcasts carry them to lane 63, which is then read by every lane.  The
// order of additions is fixed, so the result is deterministic and identical
// in all lanes.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_d<0x111, 0xF>(v);  // row_shr:1
    v += dpp_d<0x112, 0xF>(v);  // row_shr:2
    v += dpp_d<0x114, 0xF>(v);  // row_shr:4
    v += dpp_d<0x118, 0xF>(v);  // row_shr:8
    v += dpp_d<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return readlane_d(v, 63);
}

// K sums over the 64 lanes of a wavefront at once (all lanes active), every
// total returned in every lane.  The two cross-row levels are a
// reduce-scatter on the lane swaps of gfx950: swapping lanes 32-63 of one
// value with lanes 0-31 of another and adding leaves, in one register, the
// half-sums of both (one per half of the wave); the 16-lane swap of the odd
// rows of one such register with the even rows of another leaves four
// values, one per row, as 16 partial sums each.  Row shifts by 1, 2, 4, 8
// then finish every row in its lane 15.  About a third of the instructions
// of K single sums; the order of additions is fixed, so the totals are
// deterministic and identical in all lanes.
__device__ __forceinline__ void swap32_d(double& a, double& b)
{
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a),
                                                     (unsigned)__double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a),
                                                     (unsigned)__double2hiint(b), false, false);
    a = __hiloint2double((int)hi[0], (int)lo[0]);
    b = __hiloint2double((int)hi[1], (int)lo[1]);
}

__device__ __forceinline__ void swap16_d(double& a, double& b)
{
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a),
                                                     (unsigned)__double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a),
                                                     (unsigned)__double2hiint(b), false, false);
    a = __hiloint2double((int)hi[0], (int)lo[0]);
    b = __hiloint2double((int)hi[1], (int)lo[1]);
}

template <int K>
__device__ __forceinline__ void wave_sums(double (&v)[K])
{
    constexpr int K4 = (K + 3) / 4 * 4, H = K4 / 2, Q = K4 / 4;
    double w[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        // lanes 0-31: value i, lanes 32-63: value i + H, each over lane pairs
        // (l, l + 32)
        double a = i < K ? v[i] : 0.0, b = i + H < K ? v[i + H] : 0.0;
        swap32_d(a, b);
        w[i] = a + b;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // row r: value i + r Q over lane quadruples (l, l + 16, l + 32, l + 48)
        double a = w[i], b = w[i + Q];
        swap16_d(a, b);
        double x = a + b;
        x += dpp_d<0x111, 0xF>(x);  // row_shr:1
        x += dpp_d<0x112, 0xF>(x);  // row_shr:2
        x += dpp_d<0x114, 0xF>(x);  // row_shr:4
        x += dpp_d<0x118, 0xF>(x);  // row_shr:8
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (i + r * Q < K) v[i + r * Q] = readlane_d(x, 16 * r + 15);
    }
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// every thread receives the workgroup totals of its K partial sums
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red, int tid, int nt)
{
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * K + k];
        v[k] = s;
    }
}

__device__ __forceinline__ double block_min(double v, double* red, int tid, int nt)
{
    v = wave_min(v);
    const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double m = red[0];
    for (int w = 1; w < nw; ++w) m = fmin(m, red[w]);
    return m;
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane)
{
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Exclusive scan of flags over list positions [0, n) handled cyclically
// (position i by thread i % nt in round i / nt).  Calls body(i, prefix) for
// every position with its exclusive prefix; returns the total.  `wtot` holds
// one word per wave.  Rounds are processed in order, so body may move data
// downward (to prefix <= i) provided it reads before the mid barrier: the
// callable gets a flag telling which half it is in.
template <typename FlagF, typename ReadF, typename WriteF>
__device__ __forceinline__ int ordered_compact(int n, int tid, int nt, uint32_t* wtot,
                                               FlagF flag, ReadF rd, WriteF wr)
{
    const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    int base = 0;
    for (int r0 = 0; r0 < n; r0 += nt) {
        const int i = r0 + tid;
        const bool f = i < n && flag(i);
        const uint64_t m = __ballot(f);
        const int wpre = __popcll(m & lanemask_lt(lane));
        if (lane == 0) wtot[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        int off = base;
        int tot = 0;
        for (int w = 0; w < nw; ++w) {
            const int t = (int)wtot[w];
            if (w < wave) off += t;
            tot += t;
        }
        if (i < n) rd(i, f);
        __syncthreads();
        if (f) wr(i, off + wpre);
        __syncthreads();
        base += tot;
    }
    return base;
}


__device__ __forceinline__ int wrap(int i, int n) { return ((i % n) + n) % n; }

// signed cell offset along an axis; across a periodic axis the nearest image
__device__ __forceinline__ int min_image(int d, int n, bool periodic)
{
    if (!periodic) return d;
    int r = wrap(d, n);
    if (r > n - n / 2 - 1) r -= n;
    return r;
}

// basis (1, C / sqrt(theta), C^2 / (2 theta) - 3/2) of the zero-moment
// projection of an added batch
__device__ __forceinline__ void psi5(double c0, double c1, double c2, const double* U, double sq,
                                     double theta, double* psi)
{
    const double C0 = c0 - U[0], C1 = c1 - U[1], C2 = c2 - U[2];
    psi[0] = 1.0;
    psi[1] = C0 / sq;
    psi[2] = C1 / sq;
    psi[3] = C2 / sq;
    psi[4] = (C0 * C0 + C1 * C1 + C2 * C2) / (2.0 * theta) - 1.5;
}

// ---------------------------------------------------------------------------
// Step 3 for one particle: free flight by one fused multiply-add in the state
// precision; particles leaving the domain or crossing the plate's line are
// traced wall to wall in double.  Returns the destination cell (-1: the
// particle left through an open face).
// ---------------------------------------------------------------------------
template <typename real>
struct Flight {
    real px, py, c0, c1, c2;
    int clamped;
    bool gone;
};

// Full-accommodation re-emission off a surface normal to `axis`; sd = 1 when
// the surface faces the -axis direction.  Normal speed sqrt(-2 theta ln u0),
// tangential uw plus a Maxwellian from the Box-Muller pair (u1, u2).
__device__ __forceinline__ void reemit(double vel[3], int axis, int sd, double theta,
                                       const double* uw, double u0, double u1, double u2)
{
    const double vn = sqrt(-2.0 * theta * log(u0));
    const double rad = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    const int ta = axis == 0 ? 1 : 0, tb = 2;
    const double sth = sqrt(theta);
    vel[axis] = sd ? -vn : vn;
    vel[ta] = uw[ta] + sth * (rad * c);
    vel[tb] = uw[tb] + sth * (rad * s);
}

// Wall-to-wall trace of a flight of duration tl in double precision, in
// place on pos / vel.  Specular faces mirror, periodic faces wrap, diffuse
// faces and the plate re-emit (wall draws keyed by the hit number), open
// faces absorb: returns true when the particle left through one.  After 16
// hits the particle is left where it is (counted in clamped).  Inlined: an
// out-of-line call makes the caller keep its particle registers clear of the
// call-clobbered ones, which costs more registers than the trace itself.
template <int DIM, bool XB>
__device__ __forceinline__ bool trace_d(const InstDev& I, double* pos, double* vel, double tl,
                                        int src_cell, int slot, uint32_t step, int& clamped)
{
    const double lo[2] = {I.x0, I.y0}, hi[2] = {I.x1, I.y1};
    const double rest[3] = {0.0, 0.0, 0.0};
    const int a0 = DIM == 2 ? 0 : 1;
    for (int hit = 0;; ++hit) {
        if (hit == 16) {
            for (int a = a0; a < 2; ++a) {
                if (pos[a] < lo[a]) pos[a] = lo[a];
                if (pos[a] > hi[a]) pos[a] = hi[a];
            }
            ++clamped;
            return false;
        }
        double te = __builtin_inf();
        int ax = -1, sd = 0;
        for (int a = a0; a < 2; ++a) {
            double t;
            int side;
            if (vel[a] > 0.0) {
                t = (hi[a] - pos[a]) / vel[a];
                side = 1;
            } else if (vel[a] < 0.0) {
                t = (lo[a] - pos[a]) / vel[a];
                side = 0;
            } else {
                continue;
            }
            if (t < te) {
                te = t;
                ax = a;
                sd = side;
            }
        }
        bool on_plate = false;
        if (XB && DIM == 2 && I.plate) {
            // the plate's line, reached while moving towards it, inside its extent
            const double gap = I.plate_x - pos[0];
            if (gap * vel[0] > 0.0) {
                const double t = gap / vel[0];
                const double yc = pos[1] + vel[1] * t;
                if (!(yc < I.plate_ylo || yc > I.plate_yhi) && t < te) {
                    te = t;
                    on_plate = true;
                }
            }
        }
        if (!(te < tl)) {
            for (int a = a0; a < 2; ++a) pos[a] += vel[a] * tl;
            return false;
        }
        if (te < 0.0) te = 0.0;
        for (int a = a0; a < 2; ++a) pos[a] += vel[a] * te;
        tl -= te;
        uint32_t r[4];
        if (on_plate) {
            pos[0] = I.plate_x;
            draw(I, step, PUR_WALL, (uint32_t)hit, (uint32_t)src_cell, (uint32_t)slot, r);
            // back to the side it came from
            reemit(vel, 0, vel[0] > 0.0 ? 1 : 0, I.kB * I.plate_T / I.m, rest,
                   uni_d(r[0], I.prec), uni_d(r[1], I.prec), uni_d(r[2], I.prec));
            continue;
        }
        pos[ax] = sd ? hi[ax] : lo[ax];
        const int face = 2 * ax + sd;
        const int kind = I.face_kind[face];
        if (kind == 1) {
            vel[ax] = -vel[ax];
        } else if (kind == 2) {
            pos[ax] = sd ? lo[ax] : hi[ax];
        } else if (XB && kind == 3) {
            return true;
        } else {
            draw(I, step, PUR_WALL, (uint32_t)hit, (uint32_t)src_cell, (uint32_t)slot, r);
            reemit(vel, ax, sd, I.kB * I.face_T[face] / I.m, I.face_u + 3 * face,
                   uni_d(r[0], I.prec), uni_d(r[1], I.prec), uni_d(r[2], I.prec));
        }
    }
}

// trace_d of a particle held in the state precision for the whole step
template <typename real, int DIM, bool XB>
__device__ __forceinline__ Flight<real> wall_trace(const InstDev& I, real px, real py, real c0,
                                                real c1, real c2, int src_cell, int slot,
                                                uint32_t step)
{
    Flight<real> fo;
    fo.clamped = 0;
    double pos[2] = {(double)px, (double)py};
    double vel[3] = {(double)c0, (double)c1, (double)c2};
    fo.gone = trace_d<DIM, XB>(I, pos, vel, I.dt, src_cell, slot, step, fo.clamped);
    fo.px = DIM == 2 ? (real)pos[0] : px;
    fo.py = (real)pos[1];
    fo.c0 = (real)vel[0];
    fo.c1 = (real)vel[1];
    fo.c2 = (real)vel[2];
    return fo;
}

// cell of a position inside the domain (indices clamped to the grid)
template <typename real, int DIM>
__device__ __forceinline__ int cell_index(const InstDev& I, real px, real py)
{
    int iy = (int)floor(((double)py - I.y0) * I.inv_dy);
    iy = iy < 0 ? 0 : (iy > I.ny - 1 ? I.ny - 1 : iy);
    int ix = 0;
    if (DIM == 2) {
        ix = (int)floor(((double)px - I.x0) * I.inv_dx);
        ix = ix < 0 ? 0 : (ix > I.nx - 1 ? I.nx - 1 : ix);
    }
    return iy * I.nx + ix;
}

template <typename real, int DIM, bool XB>
__device__ __forceinline__ int advect(const InstDev& I, real& px, real& py, real& c0, real& c1,
                                      real& c2, int src_cell, int slot, uint32_t step, int* clamp)
{
    const real dtr = (real)I.dt;
    real np0 = px, np1;
    if (DIM == 2) np0 = fma(c0, dtr, px);
    np1 = fma(c1, dtr, py);
    bool inside = ((double)np1 >= I.y0) && ((double)np1 < I.y1);
    if (DIM == 2) inside = inside && ((double)np0 >= I.x0) && ((double)np0 < I.x1);
    if (XB && DIM == 2 && I.plate)
        inside = inside && (((double)px < I.plate_x) == ((double)np0 < I.plate_x));
    if (inside) {
        px = np0;
        py = np1;
    } else {
        const Flight<real> fl =
            wall_trace<real, DIM, XB>(I, px, py, c0, c1, c2, src_cell, slot, step);
        if (XB && fl.gone) {
            *clamp += fl.clamped;
            return -1;
        }
        px = fl.px;
        py = fl.py;
        c0 = fl.c0;
        c1 = fl.c1;
        c2 = fl.c2;
        *clamp += fl.clamped;
    }
    if (I.accel[0] != 0.0) c0 = c0 + (real)(I.accel[0] * I.dt);
    if (I.accel[1] != 0.0) c1 = c1 + (real)(I.accel[1] * I.dt);
    if (I.accel[2] != 0.0) c2 = c2 + (real)(I.accel[2] * I.dt);
    return cell_index<real, DIM>(I, px, py);
}


// Open faces (kind 3).  True when open face `face` bounds cell (ix, iy); then
// the face's area per cell (unit area in 1-D, dx or dy per unit depth in
// 2-D) and the density and theta = kT/m of the reservoir behind it (the
// second state beyond the face's split coordinate, judged at the cell centre).
template <int DIM>
__device__ __forceinline__ bool open_face(const InstDev& I, int ix, int iy, int face,
                                          double& area, double& n, double& theta)
{
    if (!((I.open_mask >> face) & 1)) return false;
    const int ax = face >> 1, sd = face & 1;
    if (DIM == 1 && ax == 0) return false;
    if (ax == 1 && iy != (sd ? I.ny - 1 : 0)) return false;
    if (ax == 0 && ix != (sd ? I.nx - 1 : 0)) return false;
    double T = I.face_T[face];
    n = I.face_n[face];
    if (DIM == 2) {
        const double tc = ax == 1 ? I.x0 + ((double)ix + 0.5) * I.dx
                                  : I.y0 + ((double)iy + 0.5) * I.dy;
        if (tc >= I.face_split[face]) {
            n = I.face_nb[face];
            T = I.face_Tb[face];
        }
        area = ax == 1 ? I.dx : I.dy;
    } else {
        area = 1.0;
    }
    theta = I.kB * T / I.m;
    return true;
}

// Particles entering cell c through open face `face` in one step: the
// effusion flux n sqrt(theta / (2 pi)) of the reservoir times area and dt
// over N_p, stochastically rounded.
template <int DIM>
__device__ __forceinline__ int inject_count(const InstDev& I, int c, int ix, int iy, int face,
                                            uint32_t step)
{
    double area, n, theta;
    if (!open_face<DIM>(I, ix, iy, face, area, n, theta)) return 0;
    const double v = n * sqrt(theta / (2.0 * M_PI)) * area * I.dt / I.Np;
    uint32_t r[4];
    draw(I, step, PUR_INJECT_CNT, (uint32_t)face, (uint32_t)c, 0u, r);
    const double u = uni_d(r[0], I.prec);
    const double fl = floor(v);
    return (int)fl + (u < v - fl ? 1 : 0);
}

// Entering particle k of cell c through open face `face` (slot: its slot in
// the cell, after the particles present): it crosses the face at a uniform
// point of the cell's share of the face and a uniform time of the step, with
// a velocity from the reservoir's flux-weighted half-range Maxwellian, and
// flies for the rest of the step (trace_d).  Returns the new cell, or -1
// when it left again through an open face.
template <typename real, int DIM>
__device__ __forceinline__ int inject_one(const InstDev& I, int c, int ix, int iy, int face,
                                          int k, int slot, uint32_t step, real& px, real& py,
                                          real& c0, real& c1, real& c2, int* clamp)
{
    double area, n, theta;
    open_face<DIM>(I, ix, iy, face, area, n, theta);
    const int ax = face >> 1, sd = face & 1;
    uint32_t r[4];
    draw(I, step, PUR_INJECT, (uint32_t)face, (uint32_t)c, (uint32_t)k, r);
    double vel[3], pos[2];
    reemit(vel, ax, sd, theta, I.face_u + 3 * face, uni_d(r[0], I.prec), uni_d(r[1], I.prec),
           uni_d(r[2], I.prec));
    const double tl = uni_d(r[3], I.prec) * I.dt;
    pos[0] = 0.0;
    if (ax == 1) {
        pos[1] = sd ? I.y1 : I.y0;
        if (DIM == 2) {
            draw(I, step, PUR_INJECT_POS, (uint32_t)face, (uint32_t)c, (uint32_t)k, r);
            pos[0] = I.x0 + ((double)ix + uni_d(r[0], I.prec)) * I.dx;
        }
    } else {
        pos[0] = sd ? I.x1 : I.x0;
        draw(I, step, PUR_INJECT_POS, (uint32_t)face, (uint32_t)c, (uint32_t)k, r);
        pos[1] = I.y0 + ((double)iy + uni_d(r[0], I.prec)) * I.dy;
    }
    int cl = 0;
    const bool gone = trace_d<DIM, true>(I, pos, vel, tl, c, slot, step, cl);
    *clamp += cl;
    if (gone) return -1;
    px = DIM == 2 ? (real)pos[0] : (real)0;
    py = (real)pos[1];
    c0 = (real)vel[0];
    c1 = (real)vel[1];
    c2 = (real)vel[2];
    return cell_index<real, DIM>(I, px, py);
}

}  // namespace usp
