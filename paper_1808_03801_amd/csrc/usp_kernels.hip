// gfx950 auxiliary kernels of the USP-ESBGK step (arXiv 1808.03801): the
// initial state (Table 2 step 1), P_ne of every cell from its own and its
// neighbours' moments (Eq. 16-18, 36), per-instance control words, the field
// record for output, and a Philox check.  The cell kernel is in usp_cell_impl.h
// (instantiated by the usp_cell_f{32,64}_{1,2}d[_xb].hip files).
#include "usp_device.h"

namespace usp {

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
        const bool use_avg = I.pne_mode == 2 && (ns_after > 0 || I.avg_init);
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
            // Eq. 18 for |u|: over max(|u|, a), or over |u| as printed (a
            // cell at rest in a velocity gradient is then fully rarefied)
            const double gu = me.lam * sqrt(g2[2]);
            const double qu = I.gll_u == 1 ? me.umag : (me.umag > a ? me.umag : a);
            const double ku = gu > 0.0 ? (qu > 0.0 ? gu / qu : INFINITY) : 0.0;
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
    if (i == 0 && B.tiers)
        for (int t = 0; t < NSHAPE; ++t) B.tiers[(size_t)t * B.tier_stride] = 0;
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
// the field record of every cell: out[c][18] (cell-major) or, with
// field_major, out[k][ncell]
__global__ void fields_out_kernel(Batch B, int which, double* out, int field_major)
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
    double r[18];
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
    for (int k = 0; k < 18; ++k) {
        if (field_major) out[(size_t)k * I.ncell + c] = r[k];
        else out[(size_t)18 * c + k] = r[k];
    }
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
template __global__ void init_kernel<float, 1>(Batch, const double*, const double*, const double*);
template __global__ void init_kernel<float, 2>(Batch, const double*, const double*, const double*);
template __global__ void init_kernel<double, 1>(Batch, const double*, const double*, const double*);
template __global__ void init_kernel<double, 2>(Batch, const double*, const double*, const double*);

}  // namespace usp
