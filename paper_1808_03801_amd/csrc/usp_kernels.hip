// gfx950 kernels of the USP-ESBGK time step (arXiv 1808.03801, Table 2).
//
// cell_kernel: one workgroup owns one cell at a time.  It gathers the cell's
// particles into LDS in canonical order, runs the relaxation of Table 2
// steps 4-8 on them (Eq. 9, 24-33, conservation, Eq. 1, 34), then adds the
// next step's f-hat particles (step 2) and advects every particle (step 3),
// writing them out grouped by destination-cell offset ("bins") together with
// a per-cell bin table.  The next launch gathers each cell's arrivals by
// reading its neighbours' bins in a fixed order, which makes the counting sort
// stable and deterministic without atomics.
//
// fields_kernel: P_ne of every cell from its own and its neighbours' moments
// (Eq. 16-18, 36).  ctl_kernel: per-instance control words.
#include "usp_device.h"

namespace usp {

template <typename real>
struct Lds {
    real* p[2];  // x (2-D), y
    real* v[3];
    real* w;
    uint32_t* key;
    uint32_t* tw;
    uint16_t* slot;
    uint16_t* bin;
    uint8_t* fate;
    double* red;
    uint32_t* hist;
    uint16_t* tiles;
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
};

template <typename real, int DIM>
__device__ __forceinline__ Lds<real> carve(unsigned char* sm, int cap, int nb, int nt)
{
    Lds<real> L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        unsigned char* q = sm + o;
        o += bytes;
        return q;
    };
    L.p[0] = DIM == 2 ? (real*)take(sizeof(real) * cap) : nullptr;
    L.p[1] = (real*)take(sizeof(real) * cap);
    for (int k = 0; k < 3; ++k) L.v[k] = (real*)take(sizeof(real) * cap);
    L.w = (real*)take(sizeof(real) * cap);
    L.key = (uint32_t*)take(4 * cap);
    L.tw = (uint32_t*)take(4 * cap);
    L.slot = (uint16_t*)take(2 * cap);
    L.bin = (uint16_t*)take(2 * cap);
    L.fate = (uint8_t*)take(cap);
    o = (o + 15) & ~(size_t)15;
    L.red = (double*)take((size_t)(nt / 64) * 24 * 8);
    L.hist = (uint32_t*)take(256 * 4);
    L.tiles = (uint16_t*)take((size_t)((cap + 63) / 64) * nb * 2);
    o = (o + 15) & ~(size_t)15;
    L.run_pre = (uint32_t*)take((size_t)(nb + 1) * 4);
    L.run_src = (uint32_t*)take((size_t)(nb + 1) * 4);
    L.run_dst = (uint32_t*)take((size_t)(nb + 1) * 4);
    L.boff = (uint32_t*)take((size_t)(nb + 1) * 4);
    o = (o + 15) & ~(size_t)15;
    L.fkey = (uint64_t*)take((size_t)FAR_LDS * 8);
    L.fent = (uint32_t*)take((size_t)FAR_LDS * 4);
    L.fpos = (uint32_t*)take((size_t)FAR_LDS * 4);
    L.fib = (uint32_t*)take((size_t)FAR_LDS * 4);
    L.fcount = (uint32_t*)take(16);
    o = (o + 15) & ~(size_t)15;
    L.sc = (double*)take(64 * 8);
    return L;
}

__device__ __forceinline__ int wrap(int i, int n) { return ((i % n) + n) % n; }

constexpr int FAR_BIN = 0xFFFF;

__device__ __forceinline__ int min_image(int d, int n, bool periodic)
{
    if (!periodic) return d;
    int r = wrap(d, n);
    if (r > n - n / 2 - 1) r -= n;
    return r;
}

// ---------------------------------------------------------------------------
// moments of list [0, n): centred (two passes) and, if RAW, raw sums; plus the
// energy total.  All threads receive the results.
// ---------------------------------------------------------------------------
template <typename real, bool RAW>
__device__ void list_moments(const Lds<real>& L, int n, int tid, int nt, double* cen,
                             double* rawout, double* E)
{
    double a[RAW ? 14 : 5];
    for (int k = 0; k < (RAW ? 14 : 5); ++k) a[k] = 0.0;
    for (int i = tid; i < n; i += nt) {
        const double w = (double)L.w[i];
        const double c0 = (double)L.v[0][i], c1 = (double)L.v[1][i], c2 = (double)L.v[2][i];
        const double cc = c0 * c0 + c1 * c1 + c2 * c2;
        a[0] += w;
        a[1] += w * c0;
        a[2] += w * c1;
        a[3] += w * c2;
        a[4] += 0.5 * w * cc;
        if (RAW) {
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
    block_sum(a, L.red, tid, nt);
    const double s0 = a[0];
    double U[3] = {0.0, 0.0, 0.0};
    if (s0 != 0.0)
        for (int k = 0; k < 3; ++k) U[k] = a[1 + k] / s0;
    double b[9];
    for (int k = 0; k < 9; ++k) b[k] = 0.0;
    for (int i = tid; i < n; i += nt) {
        const double w = (double)L.w[i];
        const double C0 = (double)L.v[0][i] - U[0], C1 = (double)L.v[1][i] - U[1];
        const double C2 = (double)L.v[2][i] - U[2];
        const double CC = C0 * C0 + C1 * C1 + C2 * C2;
        b[0] += w * C0 * C0;
        b[1] += w * C1 * C1;
        b[2] += w * C2 * C2;
        b[3] += w * C0 * C1;
        b[4] += w * C0 * C2;
        b[5] += w * C1 * C2;
        b[6] += w * CC * C0;
        b[7] += w * CC * C1;
        b[8] += w * CC * C2;
    }
    block_sum(b, L.red, tid, nt);
    cen[0] = s0;
    for (int k = 0; k < 3; ++k) cen[1 + k] = U[k];
    for (int k = 0; k < 9; ++k) cen[4 + k] = b[k];
    *E = a[4];
    if (RAW) {
        rawout[0] = a[0];
        for (int k = 0; k < 3; ++k) rawout[1 + k] = a[1 + k];
        for (int k = 0; k < 9; ++k) rawout[4 + k] = a[5 + k];
    }
}

// ---------------------------------------------------------------------------
// Zero-moment projection of the batch at [a, a + n) (optional): least-squares
// weight change that zeroes its mass, momentum and energy.
// ---------------------------------------------------------------------------
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

template <typename real>
__device__ void project_batch(const InstDev& I, const Lds<real>& L, int a, int n, const CellF& f,
                              int tid, int nt)
{
    if (n < 5) return;
    const double sq = sqrt(f.theta);
    double g[20];
    for (int k = 0; k < 20; ++k) g[k] = 0.0;
    for (int i = a + tid; i < a + n; i += nt) {
        double psi[5];
        psi5((double)L.v[0][i], (double)L.v[1][i], (double)L.v[2][i], f.U, sq, f.theta, psi);
        const double w = (double)L.w[i];
        int k = 0;
        for (int r = 0; r < 5; ++r)
            for (int s = 0; s <= r; ++s) g[k++] += psi[r] * psi[s];
        for (int r = 0; r < 5; ++r) g[15 + r] += w * psi[r];
    }
    block_sum(g, L.red, tid, nt);
    double G[5][5];
    {
        int k = 0;
        for (int r = 0; r < 5; ++r)
            for (int s = 0; s <= r; ++s) {
                G[r][s] = g[k];
                G[s][r] = g[k];
                ++k;
            }
    }
    double Lc[5][5];
    for (int r = 0; r < 5; ++r)
        for (int s = 0; s < 5; ++s) Lc[r][s] = 0.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double t = G[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= Lc[i][k] * Lc[j][k];
            if (i == j) {
                ok = ok && (t > 1e-10 * G[0][0]);
                Lc[i][i] = sqrt(t > 0.0 ? t : 1.0);
            } else {
                Lc[i][j] = t / Lc[j][j];
            }
        }
    if (!ok) return;
    double y[5], lam[5];
    for (int i = 0; i < 5; ++i) {
        double t = g[15 + i];
        for (int k = 0; k < i; ++k) t -= Lc[i][k] * y[k];
        y[i] = t / Lc[i][i];
    }
    for (int i = 4; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < 5; ++k) t -= Lc[k][i] * lam[k];
        lam[i] = t / Lc[i][i];
    }
    for (int i = a + tid; i < a + n; i += nt) {
        double psi[5];
        psi5((double)L.v[0][i], (double)L.v[1][i], (double)L.v[2][i], f.U, sq, f.theta, psi);
        double d = 0.0;
        for (int r = 0; r < 5; ++r) d += psi[r] * lam[r];
        L.w[i] = (real)((double)L.w[i] - d);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Added particles of batch 2, 4 or 7 (Eq. 25-27, Table 2), appended at
// position a.  Double-precision sampling: the stored numbers are those of a
// double computation rounded once.
// ---------------------------------------------------------------------------
template <typename real, int DIM>
__device__ int spawn_batch(const InstDev& I, const Lds<real>& L, int batch, int cell, int ix,
                           int iy, uint32_t step, const CellF& f, double pne, int a, int tid,
                           int nt, uint32_t* errbits, double* marg)
{
    if (!f.valid || !(pne > 0.0) || !(f.x > 0.0)) return 0;
    const double m1 = f.x < 1.0 ? f.x : 1.0;
    const double v = f.S0 * m1 / I.r_p;
    uint32_t r[4];
    draw(I, step, PUR_SPAWN_CNT, (uint32_t)batch, (uint32_t)cell, 0u, r);
    const double u = uni_d(r[0], I.prec);
    const double fl = floor(v);
    int na = (int)fl + (u < v - fl ? 1 : 0);
    if (marg) *marg = fmin(*marg, fabs(u - (v - fl)));
    if (a + na > I.max_ppc) {
        *errbits |= ERR_CAPACITY;
        na = I.max_ppc - a > 0 ? I.max_ppc - a : 0;
    }
    double cw = I.r_p * f.nu * pne * I.dt / 2.0;
    if (I.weight_mode == 0) cw /= m1;
    const double factor = batch == 7 ? -2.0 * (-expm1(-f.x)) / f.x : 1.0;
    const double sq = sqrt(f.theta);
    for (int k = tid; k < na; k += nt) {
        const int i = a + k;
        draw(I, step, PUR_SPAWN_POS, (uint32_t)batch, (uint32_t)cell, (uint32_t)k, r);
        const double uy = uni_d(r[0], I.prec), ux = uni_d(r[1], I.prec);
        L.p[1][i] = (real)(I.y0 + ((double)iy + uy) * I.dy);
        if (DIM == 2) L.p[0][i] = (real)(I.x0 + ((double)ix + ux) * I.dx);
        draw(I, step, PUR_SPAWN_VEL, (uint32_t)batch, (uint32_t)cell, (uint32_t)k, r);
        double z[3], C[3];
        normal3_d(r, I.prec, z);
        for (int d = 0; d < 3; ++d) {
            C[d] = sq * z[d];
            L.v[d][i] = (real)(f.U[d] + C[d]);
        }
        L.w[i] = (real)(-cw * grad_bracket(I.Pr, f, C) * factor);
    }
    __syncthreads();
    if (I.proj) project_batch(I, L, a, na, f, tid, nt);
    return na;
}

// ---------------------------------------------------------------------------
// f_G(t) sample of one reassigned particle (Table 2 step 6; Eq. 6c, 29-32)
// ---------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ int resample(const InstDev& I, const Lds<real>& L, int i, int cell,
                                        uint32_t step, const CellF& f, double pne)
{
    double t, alpha;
    if (sizeof(real) == 4) {
        const float u = uni_f(L.tw[i]);
        const float x = (float)f.x, nues = (float)(I.Pr * f.nu);
        const float tf = (float)I.dt + logf(u + (1.0f - u) * expf(-x)) / nues;
        t = (double)tf;
        alpha = (double)((float)pne + (1.0f - (float)pne) * expf(-(float)f.nu * tf));
    } else {
        const double u = uni_d(L.tw[i], I.prec);
        t = I.dt + log(u + (1.0 - u) * exp(-f.x)) / (I.Pr * f.nu);
        alpha = pne + (1.0 - pne) * exp(-f.nu * t);
    }
    const double c = (1.0 - 1.0 / I.Pr) * alpha;
    const double th = f.theta;
    const double l00 = th * (1.0 + c * f.s[0]), l11 = th * (1.0 + c * f.s[1]);
    const double l22 = th * (1.0 + c * f.s[2]);
    const double l10 = th * c * f.s[3], l20 = th * c * f.s[4], l21 = th * c * f.s[5];
    const double tiny = 1e-12 * th;
    double L00 = 0, L10 = 0, L20 = 0, L11 = 0, L21 = 0, L22 = 0;
    int fb = 0;
    if (!(l00 > tiny)) fb = 1;
    if (!fb) {
        L00 = sqrt(l00);
        L10 = l10 / L00;
        L20 = l20 / L00;
        const double d1 = l11 - L10 * L10;
        if (!(d1 > tiny)) fb = 1;
        if (!fb) {
            L11 = sqrt(d1);
            L21 = (l21 - L20 * L10) / L11;
            const double d2 = l22 - L20 * L20 - L21 * L21;
            if (!(d2 > tiny)) fb = 1;
            else L22 = sqrt(d2);
        }
    }
    if (fb) {
        L00 = L11 = L22 = sqrt(th);
        L10 = L20 = L21 = 0.0;
    }
    uint32_t r[4];
    draw(I, step, PUR_RESAMPLE, 0u, (uint32_t)cell, (uint32_t)i, r);
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
    L.v[0][i] = (real)(f.U[0] + L00 * z[0]);
    L.v[1][i] = (real)(f.U[1] + L10 * z[0] + L11 * z[1]);
    L.v[2][i] = (real)(f.U[2] + L20 * z[0] + L21 * z[1] + L22 * z[2]);
    L.w[i] = (real)1.0;
    return fb;
}

// ---------------------------------------------------------------------------
// Step 3 for one particle: free flight by one fused multiply-add in the state
// precision; particles leaving the domain are traced wall to wall in double.
// Returns the destination cell.
// ---------------------------------------------------------------------------
template <typename real, int DIM>
__device__ __forceinline__ int advect(const InstDev& I, real& px, real& py, real& c0, real& c1,
                                      real& c2, int src_cell, int slot, uint32_t step, int* clamp)
{
    const double lo[2] = {I.x0, I.y0}, hi[2] = {I.x1, I.y1};
    const real dtr = (real)I.dt;
    real np0 = px, np1;
    if (DIM == 2) np0 = fma(c0, dtr, px);
    np1 = fma(c1, dtr, py);
    bool inside = ((double)np1 >= lo[1]) && ((double)np1 < hi[1]);
    if (DIM == 2) inside = inside && ((double)np0 >= lo[0]) && ((double)np0 < hi[0]);
    if (inside) {
        px = np0;
        py = np1;
    } else {
        double pos[2] = {(double)px, (double)py};
        double vel[3] = {(double)c0, (double)c1, (double)c2};
        double tl = I.dt;
        const int a0 = DIM == 2 ? 0 : 1;
        for (int hit = 0;; ++hit) {
            if (hit == 16) {
                for (int a = a0; a < 2; ++a) {
                    if (pos[a] < lo[a]) pos[a] = lo[a];
                    if (pos[a] > hi[a]) pos[a] = hi[a];
                }
                ++*clamp;
                break;
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
            if (!(te < tl)) {
                for (int a = a0; a < 2; ++a) pos[a] += vel[a] * tl;
                break;
            }
            if (te < 0.0) te = 0.0;
            for (int a = a0; a < 2; ++a) pos[a] += vel[a] * te;
            pos[ax] = sd ? hi[ax] : lo[ax];
            tl -= te;
            const int face = 2 * ax + sd;
            const int kind = I.face_kind[face];
            if (kind == 1) {
                vel[ax] = -vel[ax];
            } else if (kind == 2) {
                pos[ax] = sd ? lo[ax] : hi[ax];
            } else {
                uint32_t r[4];
                draw(I, step, PUR_WALL, (uint32_t)hit, (uint32_t)src_cell, (uint32_t)slot, r);
                const double thw = I.kB * I.face_T[face] / I.m;
                const double u0 = uni_d(r[0], I.prec), u1 = uni_d(r[1], I.prec);
                const double u2 = uni_d(r[2], I.prec);
                const double vn = sqrt(-2.0 * thw * log(u0));
                const double rad = sqrt(-2.0 * log(u1));
                double s, c;
                sincospi(2.0 * u2, &s, &c);
                const int vi = ax;
                const int ta = vi == 0 ? 1 : 0, tb = 2;
                const double* uw = I.face_u + 3 * face;
                const double sth = sqrt(thw);
                vel[vi] = sd ? -vn : vn;
                vel[ta] = uw[ta] + sth * (rad * c);
                vel[tb] = uw[tb] + sth * (rad * s);
            }
        }
        if (DIM == 2) px = (real)pos[0];
        py = (real)pos[1];
        c0 = (real)vel[0];
        c1 = (real)vel[1];
        c2 = (real)vel[2];
    }
    if (I.accel[0] != 0.0) c0 = c0 + (real)(I.accel[0] * I.dt);
    if (I.accel[1] != 0.0) c1 = c1 + (real)(I.accel[1] * I.dt);
    if (I.accel[2] != 0.0) c2 = c2 + (real)(I.accel[2] * I.dt);
    int iy = (int)floor(((double)py - I.y0) * I.inv_dy);
    iy = iy < 0 ? 0 : (iy > I.ny - 1 ? I.ny - 1 : iy);
    int ix = 0;
    if (DIM == 2) {
        ix = (int)floor(((double)px - I.x0) * I.inv_dx);
        ix = ix < 0 ? 0 : (ix > I.nx - 1 ? I.nx - 1 : ix);
    }
    return iy * I.nx + ix;
}

// radix selection of the k-th smallest key (1-based) among selected particles
template <typename real>
__device__ uint32_t kth_key(const Lds<real>& L, int n, int k, int tid, int nt)
{
    uint32_t prefix = 0;
    int rem = k;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += nt) L.hist[b] = 0u;
        __syncthreads();
        const uint32_t hmask = shift == 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
        for (int i = tid; i < n; i += nt)
            if (L.fate[i] == 3 && (L.key[i] & hmask) == prefix)
                atomicAdd(&L.hist[(L.key[i] >> shift) & 255u], 1u);
        __syncthreads();
        if (tid < 64) {
            // lane l owns bins 4l..4l+3
            uint32_t c4[4], s = 0;
            for (int q = 0; q < 4; ++q) {
                c4[q] = L.hist[4 * tid + q];
                s += c4[q];
            }
            uint32_t incl = s;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(incl, o, 64);
                if (tid >= o) incl += t;
            }
            uint32_t excl = incl - s;
            // the bin where the running count reaches rem
            int found = -1;
            uint32_t before = 0;
            uint32_t run = excl;
            for (int q = 0; q < 4; ++q) {
                if (found < 0 && run < (uint32_t)rem && run + c4[q] >= (uint32_t)rem) {
                    found = 4 * tid + q;
                    before = run;
                }
                run += c4[q];
            }
            const uint64_t m = __ballot(found >= 0);
            const int src = __ffsll((unsigned long long)m) - 1;
            const int fb = __shfl(found, src, 64);
            const uint32_t bb = __shfl(before, src, 64);
            if (tid == 0) {
                L.sc[60] = (double)fb;
                L.sc[61] = (double)bb;
            }
        }
        __syncthreads();
        const uint32_t digit = (uint32_t)L.sc[60];
        rem -= (int)L.sc[61];
        prefix |= digit << shift;
        __syncthreads();
    }
    return prefix;
}

// ---------------------------------------------------------------------------
// The cell kernel
// ---------------------------------------------------------------------------
template <typename real, int DIM>
__device__ void process_cell(const InstDev& I, int c, int mode, int cap_lds, unsigned char* smem,
                             int tid, int nt)
{
    const int* ctl = I.ctl;
    if (ctl[CTL_ERR] != 0) return;
    const int cur = ctl[CTL_CUR];
    const uint32_t step = (uint32_t)ctl[CTL_STEP];
    const int nsamp = ctl[CTL_NSAMP];
    const int nb = I.nb;
    Lds<real> L = carve<real, DIM>(smem, cap_lds, nb, nt);
    const int ix = c % I.nx, iy = c / I.nx;
    const bool per_x = I.face_kind[0] == 2, per_y = I.face_kind[2] == 2;
    uint32_t errbits = 0;
    double* dg = I.diag ? I.diag + (size_t)c * NDIAG : nullptr;

    // ---- gather: runs of every window bin from the matching source cell
    {
        const uint32_t* tin = I.tab[cur];
        for (int b = tid; b < nb; b += nt) {
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
            uint32_t len = 0, base = 0;
            if (ok) {
                const int s = sy * I.nx + sx;
                const uint32_t* t = tin + (size_t)s * (nb + 1);
                const uint32_t a0 = t[b], a1 = t[b + 1];
                len = a1 - a0;
                base = (uint32_t)s * (uint32_t)I.cap + a0;
            }
            L.run_pre[b] = len;
            L.run_src[b] = base;
        }
        __syncthreads();
        if (tid < 64) {
            // exclusive scan of nb <= 256 run lengths by one wave
            uint32_t loc[4], s = 0;
            for (int q = 0; q < 4; ++q) {
                const int b = 4 * tid + q;
                loc[q] = b < nb ? L.run_pre[b] : 0u;
                s += loc[q];
            }
            uint32_t incl = s;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(incl, o, 64);
                if (tid >= o) incl += t;
            }
            uint32_t run = incl - s;
            for (int q = 0; q < 4; ++q) {
                const int b = 4 * tid + q;
                if (b < nb) L.run_pre[b] = run;
                run += loc[q];
            }
            if (tid == 63) L.run_pre[nb] = incl;
        }
        __syncthreads();
    }
    // far arrivals: particles that left their source cell by more than the
    // window; merged by their (source offset, slot) key
    const int nfar_all = I.far_n[cur];
    int nfc = 0;
    if (nfar_all > 0) {
        if (tid == 0) L.fcount[0] = 0u;
        __syncthreads();
        const uint32_t* fm = I.far_meta[cur];
        for (int e = tid; e < nfar_all && e < I.far_cap; e += nt)
            if ((int)fm[3 * e] == c) {
                const uint32_t k = atomicAdd(&L.fcount[0], 1u);
                if (k < (uint32_t)FAR_LDS) {
                    L.fkey[k] = ((uint64_t)fm[3 * e + 1] << 32) | (uint64_t)fm[3 * e + 2];
                    L.fent[k] = (uint32_t)e;
                }
            }
        __syncthreads();
        nfc = (int)L.fcount[0];
        if (nfc > FAR_LDS) {
            errbits |= ERR_WINDOW;
            nfc = FAR_LDS;
        }
        // rank among the far arrivals and insertion bin among the window bins
        for (int k = tid; k < nfc; k += nt) {
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
        __syncthreads();
    }
    // first destination slot of every window bin
    for (int b = tid; b < nb; b += nt) {
        uint32_t sh = 0;
        for (int k = 0; k < nfc; ++k) sh += (int)L.fib[k] <= b ? 1u : 0u;
        L.run_dst[b] = L.run_pre[b] + sh;
    }
    __syncthreads();
    const int nwin = (int)L.run_pre[nb];
    int n0 = nwin + nfc;
    if (n0 > I.max_ppc) {
        errbits |= ERR_CAPACITY;
        n0 = I.max_ppc;
    }
    {
        const real* in[6];
        for (int k = 0; k < 6; ++k) in[k] = (const real*)I.pc[cur][k];
        for (int j = tid; j < nwin; j += nt) {
            int lo = 0, hi = nb - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.run_pre[mid] <= (uint32_t)j) lo = mid;
                else hi = mid - 1;
            }
            const uint32_t off = (uint32_t)j - L.run_pre[lo];
            const size_t src = (size_t)L.run_src[lo] + off;
            const int dst = (int)(L.run_dst[lo] + off);
            if (dst >= n0) continue;
            if (DIM == 2) L.p[0][dst] = in[0][src];
            L.p[1][dst] = in[1][src];
            L.v[0][dst] = in[2][src];
            L.v[1][dst] = in[3][src];
            L.v[2][dst] = in[4][src];
            L.w[dst] = in[5][src];
        }
        if (nfc > 0) {
            const real* fin[6];
            for (int k = 0; k < 6; ++k) fin[k] = (const real*)I.far_pc[cur][k];
            for (int k = tid; k < nfc; k += nt) {
                const size_t src = L.fent[k];
                const int dst = (int)L.fpos[k];
                if (dst >= n0) continue;
                if (DIM == 2) L.p[0][dst] = fin[0][src];
                L.p[1][dst] = fin[1][src];
                L.v[0][dst] = fin[2][src];
                L.v[1][dst] = fin[3][src];
                L.v[2][dst] = fin[4][src];
                L.w[dst] = fin[5][src];
            }
        }
        __syncthreads();
    }

    int n = n0;
    double cen1[NMOM], raw1[NMOM], E1 = 0.0;
    const bool have_next_moments = (mode & (MODE_RELAX | MODE_MOMENTS)) != 0;

    if (mode & MODE_RELAX) {
        if (dg && tid == 0) {
            // the step-2 fields were written by the preceding move phase
            for (int k = 0; k < NDIAG; ++k)
                if (k != D_N2 && k != D_CLAMP && k != D_MARG_CNT2) dg[k] = 0.0;
            dg[D_NIN] = n0;
        }
        // Eq. 33: moments of f-tilde^*; totals that conservation restores
        double cen[NMOM], rawt[NMOM], E0;
        list_moments<real, true>(L, n0, tid, nt, cen, rawt, &E0);
        const double M0 = cen[0];
        const double P0[3] = {rawt[1], rawt[2], rawt[3]};
        CellF f;
        derive(I, cen, n0, f);
        if (I.jmom_mode == 1 && (int)step >= I.avg_start) {
            const double ne = avg_window(I.n_avg, nsamp);
            double A[NMOM], ma[NMOM];
            for (int k = 0; k < NMOM; ++k) {
                A[k] = (ne - 1.0) / ne * I.avgs[(size_t)k * I.ncell + c] + 1.0 / ne * rawt[k];
            }
            __syncthreads();
            if (tid == 0)
                for (int k = 0; k < NMOM; ++k) I.avgs[(size_t)k * I.ncell + c] = A[k];
            if (f.valid) {
                centred_from_raw(A, ma);
                CellF fa;
                derive(I, ma, 2, fa);
                for (int k = 0; k < 6; ++k) f.s[k] = fa.valid ? fa.s[k] : 0.0;
                for (int k = 0; k < 3; ++k) f.h[k] = fa.valid ? fa.h[k] : 0.0;
            }
        }
        int flags = 0;
        if (dg && tid == 0) {
            dg[D_M0] = M0;
            dg[D_P0X] = P0[0];
            dg[D_P0Y] = P0[1];
            dg[D_P0Z] = P0[2];
            dg[D_E0] = E0;
            dg[D_MARG_SEL] = dg[D_MARG_ROUND] = dg[D_MARG_CNT] = __builtin_inf();
        }
        if (!f.valid) {
            flags |= F_SKIP;
        } else {
            const double P = I.pcur[c];
            const double da = 1.0 + I.dt * f.nu * P / 2.0;
            const double db = 1.0 + I.dt * f.nu * I.Pr * P / 2.0;
            for (int k = 0; k < 6; ++k) f.s[k] /= da;
            for (int k = 0; k < 3; ++k) f.h[k] /= db;
            double mcnt = __builtin_inf();
            // step 4
            const int n4 = spawn_batch<real, DIM>(I, L, 4, c, ix, iy, step, f, P, n0, tid, nt,
                                                  &errbits, &mcnt);
            const int nl = n0 + n4;
            // step 5: selection
            const double psel = -expm1(-f.x);
            double ss[2] = {0.0, 0.0};
            double msel = __builtin_inf();
            for (int i = tid; i < nl; i += nt) {
                uint32_t r[4];
                draw(I, step, PUR_SELECT, 0u, (uint32_t)c, (uint32_t)i, r);
                const double u = uni_d(r[0], I.prec);
                const bool sel = u < psel;
                msel = fmin(msel, fabs(u - psel));
                L.key[i] = (r[1] & 0xFFFFF800u) | (uint32_t)i;
                L.tw[i] = r[2];
                L.fate[i] = sel ? 3 : 0;
                if (sel) {
                    ss[0] += (double)L.w[i];
                    ss[1] += 1.0;
                }
            }
            block_sum(ss, L.red, tid, nt);
            if (dg) msel = block_min(msel, L.red, tid, nt);
            const double S = ss[0];
            const int ns = (int)ss[1];
            int nusp = (int)floor(S + 0.5);
            if (nusp < 0) nusp = 0;
            if (nusp > ns) nusp = ns;
            uint32_t thr = 0;
            if (nusp > 0 && nusp < ns) thr = kth_key(L, nl, nusp, tid, nt);
            for (int i = tid; i < nl; i += nt)
                if (L.fate[i] == 3)
                    L.fate[i] = (nusp == ns || (nusp > 0 && L.key[i] <= thr)) ? 1 : 2;
            __syncthreads();
            // step 6
            double fbs[1] = {0.0};
            for (int i = tid; i < nl; i += nt)
                if (L.fate[i] == 1) fbs[0] += (double)resample(I, L, i, c, step, f, P);
            __syncthreads();
            // step 7
            const int n7 = spawn_batch<real, DIM>(I, L, 7, c, ix, iy, step, f, P, nl, tid, nt,
                                                  &errbits, &mcnt);
            // conservation
            double WrOut = 0.0, s2Out = 0.0;
            if (I.conserve_mode == 0) {
                double cs[8];
                for (int k = 0; k < 8; ++k) cs[k] = 0.0;
                for (int i = tid; i < nl + n7; i += nt) {
                    const double w = (double)L.w[i];
                    const double c0 = (double)L.v[0][i], c1 = (double)L.v[1][i];
                    const double c2 = (double)L.v[2][i];
                    if (i >= nl || L.fate[i] == 0) {
                        cs[0] += w;
                        cs[1] += w * c0;
                        cs[2] += w * c1;
                        cs[3] += w * c2;
                        cs[4] += 0.5 * w * (c0 * c0 + c1 * c1 + c2 * c2);
                    } else if (L.fate[i] == 1) {
                        cs[5] += c0;
                        cs[6] += c1;
                        cs[7] += c2;
                    }
                }
                block_sum(cs, L.red, tid, nt);
                if (nusp == 0) {
                    flags |= F_NOUSP;
                } else {
                    const double Wr = (M0 - cs[0]) / nusp;
                    WrOut = Wr;
                    if (!(Wr > 0.0)) {
                        flags |= F_FAILMASS;
                    } else {
                        const double MR = Wr * nusp;
                        double a[3], cb[3];
                        for (int k = 0; k < 3; ++k) {
                            a[k] = (P0[k] - cs[1 + k]) / MR;
                            cb[k] = cs[5 + k] / nusp;
                        }
                        double dd[1] = {0.0};
                        for (int i = tid; i < nl; i += nt)
                            if (L.fate[i] == 1) {
                                const double e0 = (double)L.v[0][i] - cb[0];
                                const double e1 = (double)L.v[1][i] - cb[1];
                                const double e2 = (double)L.v[2][i] - cb[2];
                                dd[0] += e0 * e0 + e1 * e1 + e2 * e2;
                            }
                        block_sum(dd, L.red, tid, nt);
                        const double D = dd[0];
                        const double a2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
                        double sc = 1.0;
                        if (nusp >= 2 && D > 0.0) {
                            const double s2 = (E0 - cs[4] - 0.5 * MR * a2) / (0.5 * Wr * D);
                            s2Out = s2;
                            if (s2 > 0.0) sc = sqrt(s2);
                            else flags |= F_FAILENERGY;
                        } else {
                            flags |= F_FAILENERGY;
                        }
                        for (int i = tid; i < nl; i += nt)
                            if (L.fate[i] == 1) {
                                for (int k = 0; k < 3; ++k)
                                    L.v[k][i] = (real)(a[k] + sc * ((double)L.v[k][i] - cb[k]));
                                L.w[i] = (real)Wr;
                            }
                        __syncthreads();
                    }
                }
            }
            block_sum(fbs, L.red, tid, nt);
            // compaction: survivors in slot order, then the step-7 particles
            {
                real t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0, t5 = 0;
                n = ordered_compact(
                    nl + n7, tid, nt, L.hist,
                    [&](int i) { return i >= nl || L.fate[i] != 2; },
                    [&](int i, bool f_) {
                        if (f_) {
                            if (DIM == 2) t0 = L.p[0][i];
                            t1 = L.p[1][i];
                            t2 = L.v[0][i];
                            t3 = L.v[1][i];
                            t4 = L.v[2][i];
                            t5 = L.w[i];
                        }
                    },
                    [&](int i, int dst) {
                        if (DIM == 2) L.p[0][dst] = t0;
                        L.p[1][dst] = t1;
                        L.v[0][dst] = t2;
                        L.v[1][dst] = t3;
                        L.v[2][dst] = t4;
                        L.w[dst] = t5;
                    });
            }
            if (nl + n7 > I.max_ppc) errbits |= ERR_CAPACITY;
            if (dg && tid == 0) {
                dg[D_N4] = n4;
                dg[D_PSEL] = psel;
                dg[D_MARG_SEL] = msel;
                dg[D_MARG_ROUND] = fabs(S - (floor(S) + 0.5));
                dg[D_SSEL] = S;
                dg[D_NSEL] = ns;
                dg[D_NUSP] = nusp;
                dg[D_NDEL] = ns - nusp;
                dg[D_N7] = n7;
                dg[D_CHOLFB] = fbs[0];
                dg[D_MARG_CNT] = mcnt;
                dg[D_WR] = WrOut;
                dg[D_S2] = s2Out;
            }
        }
        // step 8: moments of f^{n+1}
        list_moments<real, true>(L, n, tid, nt, cen1, raw1, &E1);
        __syncthreads();
        if (tid == 0) {
            I.cnt[c] = n;
            const double ne = avg_window(I.n_avg, nsamp);
            for (int k = 0; k < NMOM; ++k) {
                I.mom[(size_t)k * I.ncell + c] = cen1[k];
                I.raw[(size_t)k * I.ncell + c] = raw1[k];
                if ((int)step >= I.avg_start) {
                    double* A = I.avg + (size_t)k * I.ncell + c;
                    *A = (ne - 1.0) / ne * *A + 1.0 / ne * raw1[k];
                }
            }
        }
        if (dg && tid == 0) {
            dg[D_FLAGS] = flags;
            dg[D_NOUT] = n;
            dg[D_M1] = raw1[0];
            dg[D_P1X] = raw1[1];
            dg[D_P1Y] = raw1[2];
            dg[D_P1Z] = raw1[3];
            dg[D_E1] = E1;
        }
    } else if (mode & MODE_MOMENTS) {
        list_moments<real, true>(L, n, tid, nt, cen1, raw1, &E1);
        __syncthreads();
        if (tid == 0) {
            I.cnt[c] = n;
            for (int k = 0; k < NMOM; ++k) {
                I.mom[(size_t)k * I.ncell + c] = cen1[k];
                I.raw[(size_t)k * I.ncell + c] = raw1[k];
            }
        }
    }

    real* out[6];
    for (int k = 0; k < 6; ++k) out[k] = (real*)I.pc[1 - cur][k];
    uint32_t* tout = I.tab[1 - cur] + (size_t)c * (nb + 1);
    const size_t rbase = (size_t)c * I.cap;

    if (mode & MODE_MOVE) {
        // step 2 of the next time level (this one, if no relaxation ran)
        const uint32_t mstep = (mode & MODE_RELAX) ? step + 1 : step;
        double m[NMOM];
        if (have_next_moments) {
            for (int k = 0; k < NMOM; ++k) m[k] = cen1[k];
        } else {
            for (int k = 0; k < NMOM; ++k) m[k] = I.mom[(size_t)k * I.ncell + c];
        }
        CellF f;
        derive(I, m, n, f);
        const int ns_after = nsamp + (((mode & MODE_RELAX) && (int)step >= I.avg_start) ? 1 : 0);
        if (I.jmom_mode == 1 && ns_after > 0 && f.valid) {
            double A[NMOM], ma[NMOM];
            for (int k = 0; k < NMOM; ++k) A[k] = I.avg[(size_t)k * I.ncell + c];
            centred_from_raw(A, ma);
            CellF fa;
            derive(I, ma, 2, fa);
            for (int k = 0; k < 6; ++k) f.s[k] = fa.valid ? fa.s[k] : 0.0;
            for (int k = 0; k < 3; ++k) f.h[k] = fa.valid ? fa.h[k] : 0.0;
        }
        const double P2 = (mode & MODE_RELAX) ? I.pcur[c] : I.pprev[c];
        double mc2 = __builtin_inf();
        __syncthreads();
        const int n2 = spawn_batch<real, DIM>(I, L, 2, c, ix, iy, mstep, f, P2, n, tid, nt,
                                              &errbits, &mc2);
        const int nmv = n + n2;
        // step 3: advect, walls, destination bin
        int clamps = 0;
        for (int i = tid; i < nmv; i += nt) {
            real px = DIM == 2 ? L.p[0][i] : (real)0;
            real py = L.p[1][i];
            real c0 = L.v[0][i], c1 = L.v[1][i], c2 = L.v[2][i];
            const int d = advect<real, DIM>(I, px, py, c0, c1, c2, c, i, mstep, &clamps);
            if (DIM == 2) L.p[0][i] = px;
            L.p[1][i] = py;
            L.v[0][i] = c0;
            L.v[1][i] = c1;
            L.v[2][i] = c2;
            const int dx_ = d % I.nx, dy_ = d / I.nx;
            const int oy = min_image(iy - dy_, I.ny, per_y);
            const int ox = DIM == 2 ? min_image(ix - dx_, I.nx, per_x) : 0;
            int b;
            if (oy < -I.Ky || oy > I.Ky || ox < -I.Kx || ox > I.Kx) {
                b = FAR_BIN;
                const int e = atomicAdd(&I.far_n[1 - cur], 1);
                if (e < I.far_cap) {
                    uint32_t* fm = I.far_meta[1 - cur] + 3 * (size_t)e;
                    fm[0] = (uint32_t)d;
                    fm[1] = ((uint32_t)(oy + 32768) << 16) | (uint32_t)(ox + 32768);
                    fm[2] = (uint32_t)i;
                    real* const* fo = (real* const*)I.far_pc[1 - cur];
                    if (DIM == 2) fo[0][e] = px;
                    fo[1][e] = py;
                    fo[2][e] = c0;
                    fo[3][e] = c1;
                    fo[4][e] = c2;
                    fo[5][e] = L.w[i];
                } else {
                    errbits |= ERR_WINDOW;
                }
            } else {
                b = (oy + I.Ky) * I.nbx + (ox + I.Kx);
            }
            L.bin[i] = (uint16_t)b;
        }
        // stable ranks by bin: per 64-slot tile counts from wave ballots
        const int ntl = (nmv + 63) / 64;
        for (int q = tid; q < ntl * nb; q += nt) L.tiles[q] = 0;
        __syncthreads();
        const int lane = tid & 63;
        for (int r0 = 0; r0 < nmv; r0 += nt) {
            const int i = r0 + tid;
            const bool act = i < nmv;
            const int b = act ? (int)L.bin[i] : -1;
            const int tile = i >> 6;
            uint64_t rem = __ballot(act && b != FAR_BIN);
            while (rem) {
                const int leader = __ffsll((unsigned long long)rem) - 1;
                const int bv = __shfl(b, leader, 64);
                const uint64_t mm = __ballot(act && b == bv && b != FAR_BIN);
                if (lane == leader) L.tiles[tile * nb + bv] = (uint16_t)__popcll(mm);
                if (act && b == bv) L.slot[i] = (uint16_t)__popcll(mm & lanemask_lt(lane));
                rem &= ~mm;
            }
        }
        __syncthreads();
        // per-bin totals and exclusive bin offsets
        for (int b = tid; b < nb; b += nt) {
            uint32_t s = 0;
            for (int t = 0; t < ntl; ++t) s += L.tiles[t * nb + b];
            L.boff[b] = s;
        }
        __syncthreads();
        if (tid < 64) {
            uint32_t loc[4], s = 0;
            for (int q = 0; q < 4; ++q) {
                const int b = 4 * tid + q;
                loc[q] = b < nb ? L.boff[b] : 0u;
                s += loc[q];
            }
            uint32_t incl = s;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(incl, o, 64);
                if (tid >= o) incl += t;
            }
            uint32_t run = incl - s;
            for (int q = 0; q < 4; ++q) {
                const int b = 4 * tid + q;
                if (b < nb) L.boff[b] = run;
                run += loc[q];
            }
            if (tid == 63) L.boff[nb] = incl;
        }
        __syncthreads();
        // tile offsets within each bin (in place: tiles -> exclusive offsets)
        for (int b = tid; b < nb; b += nt) {
            uint32_t run = L.boff[b];
            for (int t = 0; t < ntl; ++t) {
                const uint32_t v = L.tiles[t * nb + b];
                L.tiles[t * nb + b] = (uint16_t)run;
                run += v;
            }
        }
        __syncthreads();
        for (int i = tid; i < nmv; i += nt) {
            if (L.bin[i] == FAR_BIN) continue;
            const uint32_t pos = (uint32_t)L.tiles[(i >> 6) * nb + L.bin[i]] + L.slot[i];
            L.key[pos] = (uint32_t)i;
        }
        __syncthreads();
        const int nwrite = (int)L.boff[nb];
        for (int p = tid; p < nwrite; p += nt) {
            const int i = (int)L.key[p];
            if (DIM == 2) out[0][rbase + p] = L.p[0][i];
            out[1][rbase + p] = L.p[1][i];
            out[2][rbase + p] = L.v[0][i];
            out[3][rbase + p] = L.v[1][i];
            out[4][rbase + p] = L.v[2][i];
            out[5][rbase + p] = L.w[i];
        }
        for (int b = tid; b <= nb; b += nt) tout[b] = L.boff[b];
        if (dg) {
            double cl[1] = {(double)clamps};
            block_sum(cl, L.red, tid, nt);
            if (tid == 0) {
                dg[D_N2] = n2;
                dg[D_CLAMP] = cl[0];
                dg[D_MARG_CNT2] = mc2;
            }
        }
    } else {
        // stay layout: every particle in the centre bin of its own cell
        for (int p = tid; p < n; p += nt) {
            if (DIM == 2) out[0][rbase + p] = L.p[0][p];
            out[1][rbase + p] = L.p[1][p];
            out[2][rbase + p] = L.v[0][p];
            out[3][rbase + p] = L.v[1][p];
            out[4][rbase + p] = L.v[2][p];
            out[5][rbase + p] = L.w[p];
        }
        const int centre = I.Ky * I.nbx + I.Kx;
        for (int b = tid; b <= nb; b += nt) tout[b] = b <= centre ? 0u : (uint32_t)n;
    }
    // sticky error word: one atomic per failing cell
    const uint64_t em = __ballot(errbits != 0);
    if (em) {
        uint32_t e = errbits;
        for (int o = 32; o > 0; o >>= 1) e |= __shfl_xor(e, o, 64);
        if ((tid & 63) == 0) atomicOr(&I.ctl[CTL_ERR], (int)e);
    }
}

template <typename real, int DIM>
__global__ void __launch_bounds__(256) cell_kernel(Batch B)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int g = blockIdx.x; g < B.ncells; g += gridDim.x) {
        int lo = 0, hi = B.ninst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (B.base[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        process_cell<real, DIM>(B.inst[lo], g - B.base[lo], B.mode, B.cap_lds, smem, tid, nt);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// P_ne (Eq. 16-18, lambda of Eq. 36) per cell
// ---------------------------------------------------------------------------
struct GllCell {
    int valid;
    double rho, T, umag, lam, theta;
};

__device__ void gll_cell(const InstDev& I, int c, bool use_avg, GllCell& g)
{
    double m[NMOM];
    int n = 2;
    if (use_avg) {
        double r[NMOM];
        for (int k = 0; k < NMOM; ++k) r[k] = I.avg[(size_t)k * I.ncell + c];
        centred_from_raw(r, m);
    } else {
        for (int k = 0; k < NMOM; ++k) m[k] = I.mom[(size_t)k * I.ncell + c];
        // a cell of fewer than two particles is invalid even if its weight
        // sum is positive
        n = I.cnt[c];
    }
    CellF f;
    derive(I, m, n, f);
    g.valid = f.valid;
    if (!f.valid) return;
    g.rho = f.rho;
    g.T = f.T;
    g.theta = f.theta;
    g.umag = sqrt(f.U[0] * f.U[0] + f.U[1] * f.U[1] + f.U[2] * f.U[2]);
    g.lam = 16.0 / (5.0 * sqrt(2.0 * M_PI)) * f.mu / sqrt(f.rho * f.p);
}

// mode bit 1: also copy the new P_ne into P^{n-1} (initial state)
__global__ void fields_kernel(Batch B, int init)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= B.ncells) return;
    int lo = 0, hi = B.ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.base[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    const InstDev& I = B.inst[lo];
    const int c = g - B.base[lo];
    if (I.ctl[CTL_ERR] != 0) return;
    double pn;
    if (I.pne_mode == 0) {
        pn = I.pne_fixed;
    } else {
        const int step = I.ctl[CTL_STEP];
        const int ns_after = I.ctl[CTL_NSAMP] + ((!init && step >= I.avg_start) ? 1 : 0);
        const bool use_avg = I.pne_mode == 2 && ns_after > 0;
        GllCell me;
        gll_cell(I, c, use_avg, me);
        if (!me.valid) {
            pn = 0.0;
        } else {
            const int ix = c % I.nx, iy = c / I.nx;
            double g2[3] = {0.0, 0.0, 0.0};
            for (int ax = (I.dim == 2 ? 0 : 1); ax < 2; ++ax) {
                const int nn = ax == 0 ? I.nx : I.ny;
                const int idx = ax == 0 ? ix : iy;
                const double h = ax == 0 ? I.dx : I.dy;
                const bool periodic = I.face_kind[2 * ax] == 2;
                int im = idx - 1, ip = idx + 1;
                if (periodic) {
                    im = (im + nn) % nn;
                    ip = ip % nn;
                }
                bool hm = im >= 0 && im < nn, hp = ip >= 0 && ip < nn;
                GllCell cm, cp;
                cm.valid = cp.valid = 0;
                if (hm) gll_cell(I, ax == 0 ? iy * I.nx + im : im * I.nx + ix, use_avg, cm);
                if (hp) gll_cell(I, ax == 0 ? iy * I.nx + ip : ip * I.nx + ix, use_avg, cp);
                hm = hm && cm.valid;
                hp = hp && cp.valid;
                for (int qk = 0; qk < 3; ++qk) {
                    const double qc = qk == 0 ? me.rho : (qk == 1 ? me.T : me.umag);
                    const double qm = hm ? (qk == 0 ? cm.rho : (qk == 1 ? cm.T : cm.umag)) : 0.0;
                    const double qp = hp ? (qk == 0 ? cp.rho : (qk == 1 ? cp.T : cp.umag)) : 0.0;
                    double gr = 0.0;
                    if (hm && hp) gr = (qp - qm) / (2.0 * h);
                    else if (hp) gr = (qp - qc) / h;
                    else if (hm) gr = (qc - qm) / h;
                    g2[qk] += gr * gr;
                }
            }
            const double a = sqrt(5.0 / 3.0 * me.theta);
            const double kr = me.lam * sqrt(g2[0]) / me.rho;
            const double kt = me.lam * sqrt(g2[1]) / me.T;
            const double ku = me.lam * sqrt(g2[2]) / (me.umag > a ? me.umag : a);
            double kn = kr;
            if (kt > kn) kn = kt;
            if (ku > kn) kn = ku;
            pn = exp(-kn / I.Kn_c);
        }
    }
    if (init) {
        I.pcur[c] = pn;
        I.pprev[c] = pn;
    } else {
        I.pprev[c] = I.pcur[c];
        I.pcur[c] = pn;
    }
}

// per instance: flip the particle buffer; after a relaxation also advance
// the step and the sample counter
__global__ void ctl_kernel(Batch B, int relaxed)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B.ninst) return;
    int* ctl = B.inst[i].ctl;
    if (ctl[CTL_ERR] != 0) return;
    const int oc = ctl[CTL_CUR];
    ctl[CTL_CUR] = 1 - oc;
    B.inst[i].far_n[oc] = 0;
    if (relaxed) {
        if (ctl[CTL_STEP] >= B.inst[i].avg_start) ctl[CTL_NSAMP] += 1;
        ctl[CTL_STEP] += 1;
    }
}

// ---------------------------------------------------------------------------
// Table 2 step 1: initial particles, written in the stay layout of buffer cur
// ---------------------------------------------------------------------------
template <typename real, int DIM>
__global__ void init_kernel(Batch B, const double* init_n, const double* init_u,
                            const double* init_T)
{
    const int c = blockIdx.x;
    const InstDev& I = B.inst[0];
    if (c >= I.ncell) return;
    const int cur = I.ctl[CTL_CUR];
    const int ix = c % I.nx, iy = c / I.nx;
    // particles per cell: round(n V / N_p)
    int np = (int)floor(init_n[c] * I.vcell / I.Np + 0.5);
    if (np > I.max_ppc) {
        if (threadIdx.x == 0) atomicOr(&I.ctl[CTL_ERR], ERR_CAPACITY);
        np = I.max_ppc;
    }
    const double sq = sqrt(I.kB * init_T[c] / I.m);
    real* out[6];
    for (int k = 0; k < 6; ++k) out[k] = (real*)I.pc[cur][k];
    const size_t rb = (size_t)c * I.cap;
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
        uint32_t r[4];
        draw(I, 0u, PUR_INIT_POS, 0u, (uint32_t)c, (uint32_t)k, r);
        const double uy = uni_d(r[0], I.prec), ux = uni_d(r[1], I.prec);
        out[1][rb + k] = (real)(I.y0 + ((double)iy + uy) * I.dy);
        if (DIM == 2) out[0][rb + k] = (real)(I.x0 + ((double)ix + ux) * I.dx);
        draw(I, 0u, PUR_INIT_VEL, 0u, (uint32_t)c, (uint32_t)k, r);
        double z[3];
        normal3_d(r, I.prec, z);
        for (int d = 0; d < 3; ++d) out[2 + d][rb + k] = (real)(init_u[3 * c + d] + sq * z[d]);
        out[5][rb + k] = (real)1.0;
    }
    uint32_t* t = I.tab[cur] + (size_t)c * (I.nb + 1);
    const int centre = I.Ky * I.nbx + I.Kx;
    for (int b = threadIdx.x; b <= I.nb; b += blockDim.x) t[b] = b <= centre ? 0u : (uint32_t)np;
}

// field record per cell (usp_get_fields)
__global__ void fields_out_kernel(Batch B, int which, double* out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const InstDev& I = B.inst[0];
    if (c >= I.ncell) return;
    double m[NMOM];
    if (which == 1) {
        double r[NMOM];
        for (int k = 0; k < NMOM; ++k) r[k] = I.avg[(size_t)k * I.ncell + c];
        centred_from_raw(r, m);
    } else {
        for (int k = 0; k < NMOM; ++k) m[k] = I.mom[(size_t)k * I.ncell + c];
    }
    CellF f;
    derive(I, m, which == 1 ? 2 : I.cnt[c], f);
    double* r = out + (size_t)18 * c;
    for (int k = 0; k < 18; ++k) r[k] = 0.0;
    r[0] = m[0];
    r[1] = I.F * m[0];
    for (int k = 0; k < 3; ++k) r[2 + k] = m[1 + k];
    if (f.valid) {
        r[5] = f.T;
        r[6] = f.p;
        for (int k = 0; k < 6; ++k) r[7 + k] = f.p * f.s[k];
        for (int k = 0; k < 3; ++k) r[13 + k] = f.p * f.h[k];
    }
    r[16] = I.pcur[c];
    r[17] = I.cnt[c];
}

// device Philox for checking the generator
__global__ void philox_kernel(const uint32_t* ctr, uint32_t k0, uint32_t k1, int n, uint32_t* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t r[4];
    philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1, r);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = r[k];
}

// explicit instantiations
template __global__ void cell_kernel<float, 1>(Batch);
template __global__ void cell_kernel<float, 2>(Batch);
template __global__ void cell_kernel<double, 1>(Batch);
template __global__ void cell_kernel<double, 2>(Batch);
template __global__ void init_kernel<float, 1>(Batch, const double*, const double*, const double*);
template __global__ void init_kernel<float, 2>(Batch, const double*, const double*, const double*);
template __global__ void init_kernel<double, 1>(Batch, const double*, const double*, const double*);
template __global__ void init_kernel<double, 2>(Batch, const double*, const double*, const double*);

}  // namespace usp
