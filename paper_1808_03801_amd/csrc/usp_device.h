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
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
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
    f.mu = I.mu_ref * pow(f.T / I.T_ref, I.omega);
    f.nu = f.p / f.mu;
    f.x = I.Pr * f.nu * I.dt;
    f.s[0] = (m[4] - third) / third;
    f.s[1] = (m[5] - third) / third;
    f.s[2] = (m[6] - third) / third;
    f.s[3] = m[7] / third;
    f.s[4] = m[8] / third;
    f.s[5] = m[9] / third;
    for (int k = 0; k < 3; ++k) f.h[k] = 0.5 * m[10 + k] / third;
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

// Eq. 34 window: running mean for the first n_avg samples, then exponential
__device__ __forceinline__ double avg_window(int n_avg, int n_samples)
{
    const int k = n_samples + 1;
    return (double)(k < n_avg ? k : n_avg);
}

// ---------------------------------------------------------------------------
// Wavefront / workgroup reductions (deterministic: fixed butterfly order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
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

}  // namespace usp
