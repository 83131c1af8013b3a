/*
 * CPU oracle of the USP-ESBGK per-time-step particle method (arXiv 1808.03801).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, serial, double-precision statement of the
 * method, used to check the GPU library.  Shares no code with it.
 *
 * One time step n -> n+1 is Table 2, steps 2-8, taken in this order:
 *   step 2  add particles for f-hat^n (Eq. 22, 25, 26), using the moments of
 *           f^n and the P_ne of the previous step (lag rule below);
 *   step 3  advect every particle and apply the wall conditions; then a
 *           stable counting sort of the particles by their new cell;
 *   Eq. 33  moments of f-tilde^* and the starred stress / heat flux;
 *   step 4  add particles for f^* (Eq. 24, 25, 26 with starred moments);
 *   step 5  select each particle with probability 1 - exp(-nu_ES dt) (the
 *           rate of Eq. 9); keep int(sum of selected weights) of them (Eq. 28)
 *           and delete the rest;
 *   step 6  give the kept ones velocities from f_G(t) (Eq. 6b-c) at a time t
 *           drawn from Eq. 29-30 with sigma(t) of Eq. 32, weight 1;
 *   step 7  add particles with W' = -W^* 2(1 - e^-x)/x (Eq. 27, Table 2);
 *   conservation: the reassigned particles get a common weight and a shift /
 *           scale of their velocities so that the cell's mass, momentum and
 *           energy equal those of f-tilde^* (the paper does not specify this
 *           correction; the zero collision invariants of J (Eq. 14-15) and of
 *           the ES operator make those totals the right targets).  A
 *           correction is only made where it is one: a common weight in
 *           [1/2, 2], a shift of the mean of at most 3 rms spreads of the
 *           reassigned velocities, a scale in [1/3, 3]; otherwise (with a few
 *           particles per cell, a tiny common weight would demand enormous
 *           velocities) the whole cell is corrected instead: the reassigned
 *           particles take the mass-restoring weight and every particle of
 *           the cell one shift and scale (whole_cell), and where even that is
 *           out of its window the failing part is skipped and counted;
 *   step 8  moments of f^{n+1} (Eq. 1), exponential time averaging (Eq. 34)
 *           and P_ne for the next step (Eq. 16-18 with lambda of Eq. 36).
 *
 * Readings where the paper is silent or ambiguous: P^n denotes P_ne computed
 * from the fields of f^n; steps 4-7 of step n use P^n and step 2 of step n
 * uses P^{n-1}; the count of added particles (Eq. 25) is stochastically
 * rounded; the added-particle weight is r_p (dt J/2) / (f_e min(1, nu_ES dt)),
 * which equals Eq. 26 when nu_ES dt >= 1; selection is a per-particle
 * Bernoulli trial at the rate of Eq. 9 (select_mode 1: Eq. 9's count as
 * printed, the N_s smallest rank keys); the particles kept by Eq. 28 are the
 * selected ones with the smallest random rank keys; the velocity term of
 * the GLL Knudsen number (Eq. 18) is taken over max(|u|, sqrt(5 theta / 3))
 * unless gll_u asks for |u| as printed.
 *
 * The SP-ESBGK baseline of Table 1 (scheme 1) is the same step with P_ne
 * fixed at 0 (no added particles, Eq. 33 divisors 1), N_s of Eq. 9 particles
 * (the smallest rank keys of the cell) reassigned and none deleted, and
 * velocities from the fixed target f_G of the cell through the linear map of
 * Eq. 10-11 instead of f_G(t).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed by
 * the 64-bit seed, counter = (step, purpose << 24 | sub, cell, slot).
 */
#include "usp_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Random numbers                                                            */
/* ------------------------------------------------------------------------ */

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

/* Philox4x32 with 10 rounds.  Round: multiply words 0 and 2 by the two
 * Philox multipliers, take the 64-bit products apart into high and low
 * halves, and form (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
 * lo(M0*c0)).  The key is bumped by the two Weyl constants between rounds. */
void uspo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from one 32-bit word.  Single-precision state uses the
 * 23-bit grid ((r >> 9) + 1/2) 2^-23, which is exact in float; double state
 * uses (r + 1/2) 2^-32. */
double uspo_uniform(uint32_t r, int precision)
{
    if (precision == 32) return ((double)(r >> 9) + 0.5) * 0x1p-23;
    return ((double)r + 0.5) * 0x1p-32;
}

/* Three standard normals from four uniforms by the Box-Muller transform
 * (the construction behind Eq. 10): radius sqrt(-2 ln u0) with angle 2 pi u1
 * gives z0 (cosine) and z1 (sine); radius sqrt(-2 ln u2) with angle 2 pi u3
 * gives z2. */
void uspo_normal3(const uint32_t r[4], int precision, double z[3])
{
    double u0 = uspo_uniform(r[0], precision), u1 = uspo_uniform(r[1], precision);
    double u2 = uspo_uniform(r[2], precision), u3 = uspo_uniform(r[3], precision);
    double a = sqrt(-2.0 * log(u0)), b = sqrt(-2.0 * log(u2));
    z[0] = a * cos(2.0 * M_PI * u1);
    z[1] = a * sin(2.0 * M_PI * u1);
    z[2] = b * cos(2.0 * M_PI * u3);
}

/* Eq. 30, with x = nu_ES dt: t = ln[u (e^x - 1) + 1] / nu_ES, written as
 * dt + ln(u + (1 - u) e^-x) / nu_ES, which is the same number and stays finite
 * for large x. */
double uspo_time_sample(double u, double x, double nu_es, double dt)
{
    return dt + log(u + (1.0 - u) * exp(-x)) / nu_es;
}

/* ------------------------------------------------------------------------ */
/* Data                                                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    double x, y, c[3], w;
} part;

typedef struct {
    part* p;
    int n, cap;
} plist;

static void pl_push(plist* l, part q)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 64;
        l->p = (part*)realloc(l->p, (size_t)l->cap * sizeof(part));
    }
    l->p[l->n++] = q;
}

/* diagnostics slots */
enum {
    D_NIN = 0, D_N4, D_NSEL, D_NUSP, D_NDEL, D_N7, D_NOUT, D_N2, D_SSEL, D_PSEL, D_FLAGS,
    D_CHOLFB, D_M0, D_P0X, D_P0Y, D_P0Z, D_E0, D_M1, D_P1X, D_P1Y, D_P1Z, D_E1, D_CLAMP,
    D_MARG_SEL, D_MARG_ROUND, D_MARG_CNT, D_WR, D_S2, D_MARG_CNT2, D_NINJ, D_NGONE,
    D_MARG_FACE, D_MARG_CONS
};

/* Test diagnostics of the conservation correction's branch tests: keeps in
 * *m the smallest relative gap between a tested value and its bound (a
 * value that rounding alone could move across it takes either branch). */
static void note_gap(double* m, double x, double bound)
{
    double s = fmax(fabs(x), fabs(bound));
    double r = s > 0.0 ? fabs(x - bound) / s : 0.0;
    if (r < *m) *m = r;
}

/* the same for a sign test of x = the sum of terms of total size `size` */
static void note_sign(double* m, double x, double size)
{
    double r = size > 0.0 ? fabs(x) / size : 0.0;
    if (r < *m) *m = r;
}
enum { F_SKIP = 1, F_FAILMASS = 2, F_FAILENERGY = 4, F_NOUSP = 8, F_WHOLE = 16 };

struct uspo {
    uspo_config g;
    int ncell;
    double R, F; /* gas constant kB/m; mass of one unit of weight per cell volume */
    plist* cell;
    double* mom;  /* [ncell][13] centred moments of f^n: S0, U[3], K[6], Q[3] */
    double* raw;  /* [ncell][13] raw sums of f^n: S0, S1[3], S2[6], S3[3] */
    double* avg;  /* [ncell][13] averaged raw sums of f^n (Eq. 34) */
    double* avgs; /* [ncell][13] averaged raw sums of f-tilde^* (Eq. 34) */
    double* pcur; /* P_ne^n */
    double* pprev; /* P_ne^{n-1} */
    double* diag; /* [ncell][NDIAG] */
    int n_samples, step, error;
    /* the stable sort of the last step 3: particles per cell after it, and
     * for each sorted particle its place in the sequence before it */
    int* sort_cnt;
    long long* sort_perm;
    long long sort_n;
};

static uint32_t g_key(const uspo_config* g, int i) { return i == 0 ? g->seed_lo : g->seed_hi; }

static void draw(const uspo_config* g, uint32_t step, uint32_t purpose, uint32_t sub,
                 uint32_t cell, uint32_t slot, uint32_t r[4])
{
    uint32_t ctr[4] = {step, (purpose << 24) | (sub & 0xFFFFFFu), cell, slot};
    uint32_t key[2] = {g_key(g, 0), g_key(g, 1)};
    uspo_philox4x32_10(ctr, key, r);
}

/* value as stored in the configured state precision */
static double st(const uspo_config* g, double v) { return g->precision == 32 ? (double)(float)v : v; }

static double mu_of_T(const uspo_config* g, double T) { return g->mu_ref * pow(T / g->T_ref, g->omega); }

/* ------------------------------------------------------------------------ */
/* Moments (Eq. 1)                                                           */
/* ------------------------------------------------------------------------ */

/* centred moments, two passes: S0 = sum w, U = sum w c / S0,
 * K_ij = sum w C_i C_j, Q_i = sum w |C|^2 C_i with C = c - U.
 * K order: xx, yy, zz, xy, xz, yz. */
static void moments(const part* p, int n, double m[USPO_MOM])
{
    double s0 = 0, s1[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        s0 += p[i].w;
        for (int k = 0; k < 3; ++k) s1[k] += p[i].w * p[i].c[k];
    }
    double U[3] = {0, 0, 0};
    if (s0 != 0.0)
        for (int k = 0; k < 3; ++k) U[k] = s1[k] / s0;
    double K[6] = {0, 0, 0, 0, 0, 0}, Q[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        double C[3] = {p[i].c[0] - U[0], p[i].c[1] - U[1], p[i].c[2] - U[2]};
        double w = p[i].w, C2 = C[0] * C[0] + C[1] * C[1] + C[2] * C[2];
        K[0] += w * C[0] * C[0];
        K[1] += w * C[1] * C[1];
        K[2] += w * C[2] * C[2];
        K[3] += w * C[0] * C[1];
        K[4] += w * C[0] * C[2];
        K[5] += w * C[1] * C[2];
        for (int k = 0; k < 3; ++k) Q[k] += w * C2 * C[k];
    }
    m[0] = s0;
    for (int k = 0; k < 3; ++k) m[1 + k] = U[k];
    for (int k = 0; k < 6; ++k) m[4 + k] = K[k];
    for (int k = 0; k < 3; ++k) m[10 + k] = Q[k];
}

/* raw (uncentred) sums: sum w, sum w c_i, sum w c_i c_j, sum w |c|^2 c_i */
static void raw_sums(const part* p, int n, double r[USPO_MOM])
{
    memset(r, 0, sizeof(double) * USPO_MOM);
    for (int i = 0; i < n; ++i) {
        const double* c = p[i].c;
        double w = p[i].w, c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        r[0] += w;
        for (int k = 0; k < 3; ++k) r[1 + k] += w * c[k];
        r[4] += w * c[0] * c[0];
        r[5] += w * c[1] * c[1];
        r[6] += w * c[2] * c[2];
        r[7] += w * c[0] * c[1];
        r[8] += w * c[0] * c[2];
        r[9] += w * c[1] * c[2];
        for (int k = 0; k < 3; ++k) r[10 + k] += w * c2 * c[k];
    }
}

/* centred moments from raw sums (for the averaged fields) */
static void centred_from_raw(const double r[USPO_MOM], double m[USPO_MOM])
{
    double s0 = r[0];
    double U[3] = {0, 0, 0};
    if (s0 != 0.0)
        for (int k = 0; k < 3; ++k) U[k] = r[1 + k] / s0;
    double K[6];
    K[0] = r[4] - s0 * U[0] * U[0];
    K[1] = r[5] - s0 * U[1] * U[1];
    K[2] = r[6] - s0 * U[2] * U[2];
    K[3] = r[7] - s0 * U[0] * U[1];
    K[4] = r[8] - s0 * U[0] * U[2];
    K[5] = r[9] - s0 * U[1] * U[2];
    double trR = r[4] + r[5] + r[6];
    double U2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    /* sum w c_k c_i as a full matrix */
    double R2[3][3] = {{r[4], r[7], r[8]}, {r[7], r[5], r[9]}, {r[8], r[9], r[6]}};
    double Q[3];
    for (int i = 0; i < 3; ++i) {
        double UR = U[0] * R2[0][i] + U[1] * R2[1][i] + U[2] * R2[2][i];
        Q[i] = r[10 + i] - U[i] * trR - 2.0 * UR + 2.0 * s0 * U2 * U[i];
    }
    m[0] = s0;
    for (int k = 0; k < 3; ++k) m[1 + k] = U[k];
    for (int k = 0; k < 6; ++k) m[4 + k] = K[k];
    for (int k = 0; k < 3; ++k) m[10 + k] = Q[k];
}

/* Cell scalars derived from centred moments. */
typedef struct {
    int valid;
    double S0, U[3], trK, theta, rho, p, T, mu, nu, x;
    double s[6]; /* sigma / p (trace-free, dimensionless) */
    double h[3]; /* q / p (velocity units) */
} cellf;

static void derive(const uspo* o, const double m[USPO_MOM], int n, cellf* f)
{
    const uspo_config* g = &o->g;
    memset(f, 0, sizeof(*f));
    f->S0 = m[0];
    for (int k = 0; k < 3; ++k) f->U[k] = m[1 + k];
    f->trK = m[4] + m[5] + m[6];
    f->valid = (n >= 2) && (f->S0 > 0.0) && (f->trK > 0.0);
    if (!f->valid) return;
    double third = f->trK / 3.0;
    f->theta = third / f->S0;         /* R T = p / rho */
    f->rho = o->F * f->S0;
    f->p = o->F * third;
    f->T = f->theta / o->R;
    f->mu = mu_of_T(g, f->T);
    f->nu = f->p / f->mu;             /* Eq. 4 */
    f->x = g->Pr * f->nu * g->dt;     /* nu_ES dt, nu_ES = Pr nu (Eq. 6a) */
    f->s[0] = (m[4] - third) / third;
    f->s[1] = (m[5] - third) / third;
    f->s[2] = (m[6] - third) / third;
    f->s[3] = m[7] / third;
    f->s[4] = m[8] / third;
    f->s[5] = m[9] / third;
    for (int k = 0; k < 3; ++k) f->h[k] = 0.5 * m[10 + k] / third;
}

/* Grad-13 bracket of Eq. 15 / 26 at peculiar velocity C:
 * sigma_ij C_i C_j / (2 p theta) + (2/5) Pr q_i C_i (C^2/(2 theta) - 5/2) / (p theta) */
static double grad_bracket(const uspo_config* g, const cellf* f, const double C[3])
{
    const double* s = f->s;
    double sCC = s[0] * C[0] * C[0] + s[1] * C[1] * C[1] + s[2] * C[2] * C[2] +
                 2.0 * (s[3] * C[0] * C[1] + s[4] * C[0] * C[2] + s[5] * C[1] * C[2]);
    double C2 = C[0] * C[0] + C[1] * C[1] + C[2] * C[2];
    double hC = f->h[0] * C[0] + f->h[1] * C[1] + f->h[2] * C[2];
    return sCC / (2.0 * f->theta) +
           0.4 * g->Pr * hC * (C2 / (2.0 * f->theta) - 2.5) / f->theta;
}

/* ------------------------------------------------------------------------ */
/* Adding particles: Table 2 steps 2, 4 and 7 (Eq. 25, 26, 27)               */
/* ------------------------------------------------------------------------ */

static void cell_ij(const uspo_config* g, int cell, int* ix, int* iy)
{
    *ix = cell % g->nx;
    *iy = cell / g->nx;
}

/* position uniform in the cell: lo + (index + u) * width, per resolved axis */
static void uniform_position(const uspo_config* g, int cell, const uint32_t r[4], part* q)
{
    int ix, iy;
    cell_ij(g, cell, &ix, &iy);
    double uy = uspo_uniform(r[0], g->precision), ux = uspo_uniform(r[1], g->precision);
    q->y = st(g, g->y0 + ((double)iy + uy) * g->dy);
    q->x = g->dim == 2 ? st(g, g->x0 + ((double)ix + ux) * g->dx) : 0.0;
}

/* Adds the particles of one batch (2, 4 or 7) to list L.  Count: Eq. 25,
 * N_a = S0 min(1, nu_ES dt) / r_p (S0 = rho V / (m N_p) is the cell's weight
 * sum), stochastically rounded.  Velocities: the Maxwellian f_e / rho of the
 * cell.  Weights: W = -c_w G(C) (Eq. 26) for batches 2 and 4, and
 * W' = -W 2 (1 - e^-x) / x for batch 7 (Table 2, step 7).
 * Returns the number added and the rounding margin. */
/* Zero-moment projection of one added batch (optional, not in the paper):
 * the least-squares change of the batch's weights that makes its mass,
 * momentum and energy exactly zero, which they are in expectation because J
 * has zero collision invariants (Eq. 14-15).  Basis psi = (1, C / sqrt(theta),
 * C^2 / (2 theta) - 3/2) of the stored velocities; the 5x5 Gram system is
 * solved by Cholesky.  Batches of fewer than 5 particles, or with a pivot not
 * above 1e-10 of the first diagonal entry, are left unchanged. */
static void psi_basis(const double c[3], const double U[3], double sq, double theta, double psi[5])
{
    double C[3] = {c[0] - U[0], c[1] - U[1], c[2] - U[2]};
    psi[0] = 1.0;
    psi[1] = C[0] / sq;
    psi[2] = C[1] / sq;
    psi[3] = C[2] / sq;
    psi[4] = (C[0] * C[0] + C[1] * C[1] + C[2] * C[2]) / (2.0 * theta) - 1.5;
}

static int project_batch(const uspo_config* g, part* p, int n, const double U[3], double theta)
{
    if (n < 5) return 0;
    double G[5][5], b[5], psi[5], sq = sqrt(theta);
    memset(G, 0, sizeof(G));
    memset(b, 0, sizeof(b));
    for (int k = 0; k < n; ++k) {
        psi_basis(p[k].c, U, sq, theta, psi);
        for (int i = 0; i < 5; ++i) {
            b[i] += p[k].w * psi[i];
            for (int j = 0; j < 5; ++j) G[i][j] += psi[i] * psi[j];
        }
    }
    double L[5][5];
    memset(L, 0, sizeof(L));
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) {
            double t = G[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(t > 1e-10 * G[0][0])) return -1;
                L[i][i] = sqrt(t);
            } else {
                L[i][j] = t / L[j][j];
            }
        }
    double y[5], lam[5];
    for (int i = 0; i < 5; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
        y[i] = t / L[i][i];
    }
    for (int i = 4; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < 5; ++k) t -= L[k][i] * lam[k];
        lam[i] = t / L[i][i];
    }
    for (int k = 0; k < n; ++k) {
        psi_basis(p[k].c, U, sq, theta, psi);
        double d = 0.0;
        for (int i = 0; i < 5; ++i) d += psi[i] * lam[i];
        p[k].w = st(g, p[k].w - d);
    }
    return 1;
}

static int spawn(const uspo* o, int batch, int cell, const cellf* f, double pne, plist* L,
                 double* margin)
{
    const uspo_config* g = &o->g;
    if (!f->valid || !(pne > 0.0) || !(f->x > 0.0)) return 0;
    double m1 = f->x < 1.0 ? f->x : 1.0;
    /* Eq. 25; held in [0, 1e6] (beyond every capacity) so that a blown-up
     * cell ends in the capacity error instead of an int overflow */
    double v = fmin(fmax(f->S0 * m1 / g->r_p, 0.0), 1.0e6);
    uint32_t r[4];
    draw(g, (uint32_t)o->step, PUR_SPAWN_CNT, (uint32_t)batch, (uint32_t)cell, 0, r);
    double u = uspo_uniform(r[0], g->precision);
    double fl = floor(v);
    int na = (int)fl + (u < v - fl ? 1 : 0);
    if (margin) {
        double mg = fabs(u - (v - fl));
        if (mg < *margin) *margin = mg;
    }
    double cw = g->r_p * f->nu * pne * g->dt / 2.0;
    if (g->weight_mode == 0) cw /= m1;
    double factor = 1.0;
    if (batch == 7) factor = -2.0 * (-expm1(-f->x)) / f->x;
    double sq = sqrt(f->theta);
    for (int k = 0; k < na; ++k) {
        part q;
        draw(g, (uint32_t)o->step, PUR_SPAWN_POS, (uint32_t)batch, (uint32_t)cell, (uint32_t)k, r);
        uniform_position(g, cell, r, &q);
        draw(g, (uint32_t)o->step, PUR_SPAWN_VEL, (uint32_t)batch, (uint32_t)cell, (uint32_t)k, r);
        double z[3], C[3];
        uspo_normal3(r, g->precision, z);
        for (int d = 0; d < 3; ++d) {
            C[d] = sq * z[d];
            q.c[d] = st(g, f->U[d] + C[d]);
        }
        q.w = st(g, -cw * grad_bracket(g, f, C) * factor);
        pl_push(L, q);
    }
    if (g->spawn_projection == 1) project_batch(g, L->p + (L->n - na), na, f->U, f->theta);
    return na;
}

/* ------------------------------------------------------------------------ */
/* Step 3: advection and walls                                               */
/* ------------------------------------------------------------------------ */

/* Where a flight ends next to a face that two cells share (an interior
 * face, or a periodic pair), its rounding decides which of them receives
 * the particle.  Keeps, in both cells, the smallest distance of a landing
 * point in cell d to such a face (test diagnostics only: the step does not
 * read it).  Walls are not such faces: a landing point at a wall stays in
 * its cell. */
static void note_face_margin(const uspo_config* g, double* diag, int d, const part* q)
{
    int ix = d % g->nx, iy = d / g->nx;
    double best = INFINITY;
    int other = -1;
    for (int a = g->dim == 2 ? 0 : 1; a < 2; ++a) {
        double pos = a == 0 ? q->x : q->y, org = a == 0 ? g->x0 : g->y0;
        double h = a == 0 ? g->dx : g->dy;
        int i = a == 0 ? ix : iy, n = a == 0 ? g->nx : g->ny;
        int periodic = g->face_kind[2 * a] == 2;
        for (int sd = 0; sd < 2; ++sd) {
            int j = i + (sd ? 1 : -1);
            if (j < 0 || j >= n) {
                if (!periodic || n == 1) continue;
                j = (j + n) % n;
            }
            double dist = fabs(pos - (org + (i + sd) * h));
            if (dist < best) {
                best = dist;
                other = a == 0 ? iy * g->nx + j : j * g->nx + ix;
            }
        }
    }
    if (other < 0) return;
    double* m0 = diag + (size_t)USPO_NDIAG * d + D_MARG_FACE;
    double* m1 = diag + (size_t)USPO_NDIAG * other + D_MARG_FACE;
    if (best < *m0) *m0 = best;
    if (best < *m1) *m1 = best;
}

static int cell_of(const uspo_config* g, double x, double y)
{
    int iy = (int)floor((y - g->y0) * g->inv_dy);
    if (iy < 0) iy = 0;
    if (iy > g->ny - 1) iy = g->ny - 1;
    int ix = 0;
    if (g->dim == 2) {
        ix = (int)floor((x - g->x0) * g->inv_dx);
        if (ix < 0) ix = 0;
        if (ix > g->nx - 1) ix = g->nx - 1;
    }
    return iy * g->nx + ix;
}

/* Diffuse re-emission with full accommodation from a wall or an open face:
 * normal speed sqrt(-2 theta ln u0) away from the surface (side sd = 1 means
 * the surface faces the -axis direction), tangential velocity uw plus a
 * Maxwellian at theta from the Box-Muller pair of (u1, u2). */
static void reemit(double vel[3], int axis, int sd, double theta, const double uw[3], double u0,
                   double u1, double u2)
{
    double vn = sqrt(-2.0 * theta * log(u0));
    double rad = sqrt(-2.0 * log(u1));
    double z0 = rad * cos(2.0 * M_PI * u2), z1 = rad * sin(2.0 * M_PI * u2);
    int ta = axis == 0 ? 1 : 0, tb = 2;
    vel[axis] = sd ? -vn : vn;
    vel[ta] = uw[ta] + sqrt(theta) * z0;
    vel[tb] = uw[tb] + sqrt(theta) * z1;
}

/* Time for a particle at pos moving with vel to reach the internal plate, or
 * infinity when it does not reach it (moving along or away from the plate's
 * line, or crossing the line outside the plate's extent). */
static double plate_time(const uspo_config* g, const double pos[2], const double vel[3])
{
    if (!g->plate) return INFINITY;
    double gap = g->plate_x - pos[0];
    if (!(gap * vel[0] > 0.0)) return INFINITY;
    double t = gap / vel[0];
    double yc = pos[1] + vel[1] * t;
    if (yc < g->plate_ylo || yc > g->plate_yhi) return INFINITY;
    return t;
}

/* Wall-to-wall flight of duration tl in double precision.  Specular faces
 * mirror the normal velocity, periodic faces wrap, diffuse faces and the
 * plate re-emit the particle (reemit, wall draws keyed by the hit number)
 * for the rest of the flight, open faces absorb it.  After 16 hits the
 * particle is left where it is (counted in *clamped).  Returns 1 when the
 * particle left through an open face. */
static int trace(const uspo_config* g, double pos[2], double vel[3], double tl, int src_cell,
                 int slot, int step, int* clamped)
{
    double lo[2] = {g->x0, g->y0}, hi[2] = {g->x1, g->y1};
    int a_first = g->dim == 2 ? 0 : 1;
    for (int hit = 0;; ++hit) {
        if (hit == 16) {
            for (int a = a_first; a < 2; ++a) {
                if (pos[a] < lo[a]) pos[a] = lo[a];
                if (pos[a] > hi[a]) pos[a] = hi[a];
            }
            ++*clamped;
            return 0;
        }
        double te = INFINITY;
        int ax = -1, sd = 0;
        for (int a = a_first; a < 2; ++a) {
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
        double tp = plate_time(g, pos, vel);
        int on_plate = tp < te;
        if (on_plate) te = tp;
        if (!(te < tl)) {
            for (int a = a_first; a < 2; ++a) pos[a] += vel[a] * tl;
            return 0;
        }
        if (te < 0.0) te = 0.0;
        for (int a = a_first; a < 2; ++a) pos[a] += vel[a] * te;
        tl -= te;
        uint32_t r[4];
        if (on_plate) {
            static const double rest[3] = {0.0, 0.0, 0.0};
            pos[0] = g->plate_x;
            draw(g, (uint32_t)step, PUR_WALL, (uint32_t)hit, (uint32_t)src_cell, (uint32_t)slot,
                 r);
            /* back to the side it came from */
            reemit(vel, 0, vel[0] > 0.0, g->kB * g->plate_T / g->m, rest,
                   uspo_uniform(r[0], g->precision), uspo_uniform(r[1], g->precision),
                   uspo_uniform(r[2], g->precision));
            continue;
        }
        pos[ax] = sd ? hi[ax] : lo[ax];
        int face = 2 * ax + sd;
        int kind = g->face_kind[face];
        if (kind == 1) {
            vel[ax] = -vel[ax];
        } else if (kind == 2) {
            pos[ax] = sd ? lo[ax] : hi[ax];
        } else if (kind == 3) {
            return 1;
        } else {
            draw(g, (uint32_t)step, PUR_WALL, (uint32_t)hit, (uint32_t)src_cell, (uint32_t)slot,
                 r);
            reemit(vel, ax, sd, g->kB * g->face_T[face] / g->m, g->face_u + 3 * face,
                   uspo_uniform(r[0], g->precision), uspo_uniform(r[1], g->precision),
                   uspo_uniform(r[2], g->precision));
        }
    }
}

/* Moves one particle for dt.  A particle that stays inside (and does not
 * cross the plate's line) moves by one fused multiply-add in the state
 * precision; any other is traced in double precision (trace).  A body
 * acceleration (the Poiseuille drive) adds a dt to the velocity afterwards.
 * Returns the new cell, or -1 when the particle left through an open face. */
static int advect(const uspo_config* g, part* q, int src_cell, int slot, int step, int* clamped)
{
    double lo[2] = {g->x0, g->y0}, hi[2] = {g->x1, g->y1};
    int a_first = g->dim == 2 ? 0 : 1;
    double np[2];
    if (g->precision == 32) {
        np[0] = g->dim == 2 ? (double)fmaf((float)q->c[0], (float)g->dt, (float)q->x) : q->x;
        np[1] = (double)fmaf((float)q->c[1], (float)g->dt, (float)q->y);
    } else {
        np[0] = g->dim == 2 ? fma(q->c[0], g->dt, q->x) : q->x;
        np[1] = fma(q->c[1], g->dt, q->y);
    }
    int inside = 1;
    for (int a = a_first; a < 2; ++a)
        if (!(np[a] >= lo[a] && np[a] < hi[a])) inside = 0;
    if (g->plate && ((q->x < g->plate_x) != (np[0] < g->plate_x))) inside = 0;
    if (inside) {
        q->x = np[0];
        q->y = np[1];
    } else {
        double pos[2] = {q->x, q->y}, vel[3] = {q->c[0], q->c[1], q->c[2]};
        if (trace(g, pos, vel, g->dt, src_cell, slot, step, clamped)) return -1;
        q->x = g->dim == 2 ? st(g, pos[0]) : q->x;
        q->y = st(g, pos[1]);
        for (int k = 0; k < 3; ++k) q->c[k] = st(g, vel[k]);
    }
    for (int k = 0; k < 3; ++k)
        if (g->accel[k] != 0.0) q->c[k] = st(g, q->c[k] + st(g, g->accel[k] * g->dt));
    return cell_of(g, q->x, q->y);
}

/* Open faces (kind 3).  Does open face `face` bound cell c?  If so, *area is
 * the face's area per cell (unit area in 1-D, dx or dy per unit depth in
 * 2-D) and *n, *theta the state of the reservoir behind it. */
static int open_face_of(const uspo_config* g, int c, int face, double* area, double* n,
                        double* theta)
{
    if (g->face_kind[face] != 3) return 0;
    int ax = face / 2, sd = face % 2, ix, iy;
    if (g->dim == 1 && ax == 0) return 0;
    cell_ij(g, c, &ix, &iy);
    if (ax == 1 && iy != (sd ? g->ny - 1 : 0)) return 0;
    if (ax == 0 && ix != (sd ? g->nx - 1 : 0)) return 0;
    double tc = 0.0, T = g->face_T[face];
    *n = g->face_n[face];
    if (g->dim == 2) {
        tc = ax == 1 ? g->x0 + ((double)ix + 0.5) * g->dx : g->y0 + ((double)iy + 0.5) * g->dy;
        if (tc >= g->face_split[face]) {
            *n = g->face_nb[face];
            T = g->face_Tb[face];
        }
        *area = ax == 1 ? g->dx : g->dy;
    } else {
        *area = 1.0;
    }
    *theta = g->kB * T / g->m;
    return 1;
}

/* Number of particles entering cell c through open face `face` in one step:
 * the one-sided flux of a gas at rest, n sqrt(theta / (2 pi)) per unit area
 * and time (the kinetic-theory effusion rate), times area and dt over N_p,
 * stochastically rounded. */
static int inject_count(const uspo_config* g, int step, int c, int face)
{
    double area, n, theta;
    if (!open_face_of(g, c, face, &area, &n, &theta)) return 0;
    double v = n * sqrt(theta / (2.0 * M_PI)) * area * g->dt / g->Np;
    uint32_t r[4];
    draw(g, (uint32_t)step, PUR_INJECT_CNT, (uint32_t)face, (uint32_t)c, 0, r);
    double u = uspo_uniform(r[0], g->precision);
    double fl = floor(v);
    return (int)fl + (u < v - fl ? 1 : 0);
}

/* Entering particle k of cell c through open face `face` (slot = its slot in
 * the cell, after the particles present): it crosses the face at a uniform
 * point of the cell's face segment, at a uniform time of the step, with a
 * velocity from the flux-weighted half-range Maxwellian of the reservoir
 * (normal speed sqrt(-2 theta ln u), tangential face velocity plus a
 * Maxwellian), weight 1, and flies for the rest of the step (trace).
 * Returns the new cell or -1 (it left again through an open face). */
static int inject_one(const uspo_config* g, int step, int c, int face, int k, int slot, part* q,
                      int* clamped)
{
    double area, n, theta;
    open_face_of(g, c, face, &area, &n, &theta);
    int ax = face / 2, sd = face % 2, ix, iy;
    cell_ij(g, c, &ix, &iy);
    uint32_t r[4];
    draw(g, (uint32_t)step, PUR_INJECT, (uint32_t)face, (uint32_t)c, (uint32_t)k, r);
    double vel[3], pos[2];
    reemit(vel, ax, sd, theta, g->face_u + 3 * face, uspo_uniform(r[0], g->precision),
           uspo_uniform(r[1], g->precision), uspo_uniform(r[2], g->precision));
    double tl = uspo_uniform(r[3], g->precision) * g->dt;
    pos[0] = 0.0;
    if (ax == 1) {
        pos[1] = sd ? g->y1 : g->y0;
        if (g->dim == 2) {
            draw(g, (uint32_t)step, PUR_INJECT_POS, (uint32_t)face, (uint32_t)c, (uint32_t)k, r);
            pos[0] = g->x0 + ((double)ix + uspo_uniform(r[0], g->precision)) * g->dx;
        }
    } else {
        pos[0] = sd ? g->x1 : g->x0;
        draw(g, (uint32_t)step, PUR_INJECT_POS, (uint32_t)face, (uint32_t)c, (uint32_t)k, r);
        pos[1] = g->y0 + ((double)iy + uspo_uniform(r[0], g->precision)) * g->dy;
    }
    if (trace(g, pos, vel, tl, c, slot, step, clamped)) return -1;
    q->x = g->dim == 2 ? st(g, pos[0]) : 0.0;
    q->y = st(g, pos[1]);
    for (int d = 0; d < 3; ++d) q->c[d] = st(g, vel[d]);
    q->w = 1.0;
    return cell_of(g, q->x, q->y);
}

/* ------------------------------------------------------------------------ */
/* Stable counting sort by new cell.  Canonical order inside a cell: by the  */
/* source cell's displacement from the destination (row-major, minimal image */
/* across periodic faces), then by the particle's slot in its source cell.   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int dest, dy, dx, slot;
    long long pre; /* place in the sequence before the sort */
    part q;
} sentry;

static int cmp_entry(const void* a, const void* b)
{
    const sentry* p = (const sentry*)a;
    const sentry* r = (const sentry*)b;
    if (p->dest != r->dest) return p->dest < r->dest ? -1 : 1;
    if (p->dy != r->dy) return p->dy < r->dy ? -1 : 1;
    if (p->dx != r->dx) return p->dx < r->dx ? -1 : 1;
    if (p->slot != r->slot) return p->slot < r->slot ? -1 : 1;
    return 0;
}

static int min_image(int delta, int n, int periodic)
{
    if (!periodic) return delta;
    int d = ((delta % n) + n) % n;
    if (d > n - n / 2 - 1) d -= n;
    return d;
}

/* ------------------------------------------------------------------------ */
/* Steps 4-8 for one cell                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int sel;      /* selected in step 5 */
    int fate;     /* 0 kept as is, 1 reassigned, 2 deleted */
    uint32_t rank;
    double ut;
} selinfo;

static int cmp_rank(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void totals(const part* p, int n, double* M, double P[3], double* E)
{
    *M = 0;
    P[0] = P[1] = P[2] = 0;
    *E = 0;
    for (int i = 0; i < n; ++i) {
        double w = p[i].w;
        *M += w;
        for (int k = 0; k < 3; ++k) P[k] += w * p[i].c[k];
        *E += 0.5 * w * (p[i].c[0] * p[i].c[0] + p[i].c[1] * p[i].c[1] + p[i].c[2] * p[i].c[2]);
    }
}

/* f_G(t) sample for one reassigned particle (Table 2 step 6, Eq. 6b-c, 29-32):
 * lambda(t) = theta (I + (1 - 1/Pr) alpha(t) s*), alpha = P + (1-P) e^{-nu t};
 * velocity u* + L z with L the Cholesky factor of lambda.  A pivot not above
 * 1e-12 theta falls back to the isotropic factor sqrt(theta) I. */
/* The linear map of Eq. 10-11: a Maxwellian thermal velocity at the cell's
 * temperature mapped by S = I - (1 - Pr) / (2 Pr) a (p_ij / (rho theta) - I),
 * where p_ij / (rho theta) - I = sigma / p; c = u + sqrt(theta) S z.  a = 1
 * is SP-ESBGK's fixed target (Table 1, steps 3-4); a = alpha of Eq. 32 maps
 * to USP-ESBGK's f_G(t) with es_sampler 1 (the covariance theta S S^T equals
 * the target's to first order in sigma / p). */
static void resample_linear(const uspo* o, const cellf* f, double a, int cell, int slot,
                            part* q)
{
    const uspo_config* g = &o->g;
    double k = (1.0 - g->Pr) / (2.0 * g->Pr) * a;
    double S00 = 1.0 - k * f->s[0], S11 = 1.0 - k * f->s[1], S22 = 1.0 - k * f->s[2];
    double S01 = -k * f->s[3], S02 = -k * f->s[4], S12 = -k * f->s[5];
    uint32_t r[4];
    draw(g, (uint32_t)o->step, PUR_RESAMPLE, 0, (uint32_t)cell, (uint32_t)slot, r);
    double z[3];
    uspo_normal3(r, g->precision, z);
    double sq = sqrt(f->theta);
    q->c[0] = st(g, f->U[0] + sq * (S00 * z[0] + S01 * z[1] + S02 * z[2]));
    q->c[1] = st(g, f->U[1] + sq * (S01 * z[0] + S11 * z[1] + S12 * z[2]));
    q->c[2] = st(g, f->U[2] + sq * (S02 * z[0] + S12 * z[1] + S22 * z[2]));
    q->w = 1.0;
}

static int resample(const uspo* o, const cellf* f, double pne, int cell, int slot, double ut,
                    part* q)
{
    const uspo_config* g = &o->g;
    if (g->scheme == 1) {
        resample_linear(o, f, 1.0, cell, slot, q);
        return 0;
    }
    double alpha;
    if (g->es_mode == 1) {
        /* the expectation of alpha(t) over the Eq. 29-30 time distribution,
         * density nu_ES e^{nu_ES t} / (e^{nu_ES dt} - 1) on [0, dt]:
         * E e^{-nu t} = Pr / (Pr - 1) (e^{(Pr - 1) nu dt} - 1) / (e^{Pr nu dt} - 1) */
        double Pr = g->Pr, y = f->nu * g->dt;
        double m = Pr / (Pr - 1.0) * expm1((Pr - 1.0) * y) / expm1(Pr * y);
        alpha = pne + (1.0 - pne) * m;
    } else {
        double t = uspo_time_sample(ut, f->x, g->Pr * f->nu, g->dt);
        alpha = pne + (1.0 - pne) * exp(-f->nu * t);
    }
    if (g->es_sampler == 1) {
        resample_linear(o, f, alpha, cell, slot, q);
        return 0;
    }
    double c = (1.0 - 1.0 / g->Pr) * alpha;
    double th = f->theta;
    double l00 = th * (1.0 + c * f->s[0]), l11 = th * (1.0 + c * f->s[1]);
    double l22 = th * (1.0 + c * f->s[2]);
    double l10 = th * c * f->s[3], l20 = th * c * f->s[4], l21 = th * c * f->s[5];
    double tiny = 1e-12 * th;
    double L00, L10, L20, L11, L21, L22;
    int fb = 0;
    if (!(l00 > tiny)) fb = 1;
    if (!fb) {
        L00 = sqrt(l00);
        L10 = l10 / L00;
        L20 = l20 / L00;
        double d1 = l11 - L10 * L10;
        if (!(d1 > tiny)) fb = 1;
        if (!fb) {
            L11 = sqrt(d1);
            L21 = (l21 - L20 * L10) / L11;
            double d2 = l22 - L20 * L20 - L21 * L21;
            if (!(d2 > tiny)) fb = 1;
            else L22 = sqrt(d2);
        }
    }
    if (fb) {
        L00 = L11 = L22 = sqrt(th);
        L10 = L20 = L21 = 0.0;
    }
    uint32_t r[4];
    draw(g, (uint32_t)o->step, PUR_RESAMPLE, 0, (uint32_t)cell, (uint32_t)slot, r);
    double z[3];
    uspo_normal3(r, g->precision, z);
    q->c[0] = st(g, f->U[0] + L00 * z[0]);
    q->c[1] = st(g, f->U[1] + L10 * z[0] + L11 * z[1]);
    q->c[2] = st(g, f->U[2] + L20 * z[0] + L21 * z[1] + L22 * z[2]);
    q->w = 1.0;
    return fb;
}

/* Eq. 34 with n_a = min(k + 1, n_avg) for the k-th sample (k from 0): the
 * plain running mean of the samples until n_avg of them exist, then the
 * exponentially weighted average with n_a = n_avg. */
static double avg_window(const uspo_config* g, int n_samples)
{
    int k = n_samples + 1;
    if (g->avg_init) return (double)g->n_avg;
    return (double)(k < g->n_avg ? k : g->n_avg);
}

/* Stress and heat flux that build the added particles and f_G: those of
 * the cell (instantaneous), or, with time-averaged moments, those of the
 * Eq. 34 average (zero where the average is not a valid state). */
static void use_averaged_sh(const uspo* o, const double* avg_raw, cellf* f)
{
    double m[USPO_MOM];
    centred_from_raw(avg_raw, m);
    cellf fa;
    derive(o, m, 2, &fa);
    for (int k = 0; k < 6; ++k) f->s[k] = fa.valid ? fa.s[k] : 0.0;
    for (int k = 0; k < 3; ++k) f->h[k] = fa.valid ? fa.h[k] : 0.0;
}

/* Conservation where the reassigned particles alone cannot carry it (a
 * common weight outside [1/2, 2], or a shift / scale outside its window):
 * the reassigned particles take the common weight W_r that restores the
 * cell's mass (any W_r > 0), and then every particle that stays in the cell
 * (survivors, reassigned, step-7 particles) gets one shift and scale,
 *   c -> P0 / M0 + s (c - u),   s^2 = (E0 - |P0|^2 / (2 M0)) / K,
 * with u and K the mean velocity and thermal energy of that set, so that the
 * cell's momentum and energy equal those of f-tilde^*.  Made where it is a
 * correction: at least two reassigned particles (with one, the cell keeps
 * the one-particle change), W_r > 0, K > 0, a shift of at most 3 rms
 * thermal speeds and s^2 in [1/4, 4] (a wider scale, with K a difference of
 * the positive- and negative-weight particles' energies, can spread a cell's
 * velocities far enough to destabilise it at a few dozen particles per
 * cell).  Returns 1
 * if made, 0 (nothing changed) otherwise.  Mr, Pr, Er: mass, momentum and
 * energy of the survivors and the step-7 particles. */
static int whole_cell(const uspo* o, plist* L, const selinfo* si, int nl, plist* L7, int nusp,
                      double M0, const double P0[3], double E0, double Mr, const double Pr[3],
                      double Er, double* gap)
{
    const uspo_config* g = &o->g;
    double Wr = (M0 - Mr) / nusp;
    double sc[3] = {0, 0, 0}, sq = 0.0;
    for (int i = 0; i < nl; ++i)
        if (si[i].fate == 1)
            for (int k = 0; k < 3; ++k) {
                sc[k] += L->p[i].c[k];
                sq += L->p[i].c[k] * L->p[i].c[k];
            }
    int ok = nusp >= 2 && Wr > 0.0;
    double M = Mr + Wr * nusp, u[3], a[3], u2 = 0.0, a2 = 0.0, du2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        u[k] = (Pr[k] + Wr * sc[k]) / M;
        a[k] = P0[k] / M0;
        u2 += u[k] * u[k];
        a2 += a[k] * a[k];
        du2 += (a[k] - u[k]) * (a[k] - u[k]);
    }
    double K = Er + 0.5 * Wr * sq - 0.5 * M * u2;
    double s2 = (E0 - 0.5 * M0 * a2) / K;
    note_sign(gap, M0 - Mr, fabs(M0) + fabs(Mr));
    note_sign(gap, M, fabs(Mr) + fabs(Wr * nusp));
    note_sign(gap, K, fabs(Er) + fabs(0.5 * Wr * sq) + fabs(0.5 * M * u2));
    if (K > 0.0 && M > 0.0) {
        note_gap(gap, du2, 9.0 * 2.0 * K / M);
        note_gap(gap, s2, 0.25);
        note_gap(gap, s2, 4.0);
    }
    ok = ok && M > 0.0 && K > 0.0 && du2 <= 9.0 * 2.0 * K / M && s2 >= 0.25 && s2 <= 4.0;
    if (!ok) return 0;
    double s = sqrt(s2);
    for (int pass = 0; pass < 2; ++pass) {
        part* pp = pass == 0 ? L->p : L7->p;
        int np = pass == 0 ? nl : L7->n;
        for (int i = 0; i < np; ++i) {
            if (pass == 0 && si[i].fate == 2) continue;
            part* q = &pp[i];
            if (pass == 0 && si[i].fate == 1) q->w = st(g, Wr);
            for (int k = 0; k < 3; ++k) q->c[k] = st(g, a[k] + s * (q->c[k] - u[k]));
        }
    }
    return 1;
}

static void relax_cell(uspo* o, int d, plist* L, double* dg)
{
    const uspo_config* g = &o->g;
    int n0 = L->n;
    dg[D_NIN] = n0;
    dg[D_MARG_SEL] = dg[D_MARG_ROUND] = dg[D_MARG_CNT] = dg[D_MARG_CONS] = INFINITY;
    double mom[USPO_MOM];
    moments(L->p, n0, mom);
    double M0, P0[3], E0;
    totals(L->p, n0, &M0, P0, &E0);
    dg[D_M0] = M0;
    dg[D_P0X] = P0[0]; dg[D_P0Y] = P0[1]; dg[D_P0Z] = P0[2];
    dg[D_E0] = E0;
    cellf f;
    derive(o, mom, n0, &f);
    if (g->jmom_mode == 1 && o->step >= g->avg_start) {
        double r[USPO_MOM];
        raw_sums(L->p, n0, r);
        double* A = o->avgs + (size_t)USPO_MOM * d;
        double ne = avg_window(g, o->n_samples);
        for (int k = 0; k < USPO_MOM; ++k) A[k] = (ne - 1.0) / ne * A[k] + 1.0 / ne * r[k];
        if (f.valid) use_averaged_sh(o, A, &f);
    }
    int flags = 0;
    plist L7 = {0, 0, 0};
    if (!f.valid) {
        flags |= F_SKIP;
    } else {
        double P = o->pcur[d];
        /* Eq. 33: stress and heat flux of f^* from those of f-tilde^* */
        double da = 1.0 + g->dt * f.nu * P / 2.0;
        double db = 1.0 + g->dt * f.nu * g->Pr * P / 2.0;
        for (int k = 0; k < 6; ++k) f.s[k] /= da;
        for (int k = 0; k < 3; ++k) f.h[k] /= db;

        /* step 4 */
        int n4 = spawn(o, 4, d, &f, P, L, &dg[D_MARG_CNT]);
        dg[D_N4] = n4;
        int nl = L->n;
        if (nl > g->max_ppc) o->error = -3;

        /* step 5: Bernoulli selection with probability 1 - exp(-nu_ES dt);
         * SP-ESBGK: every particle is a candidate and Eq. 9 fixes how many
         * of them are reassigned (S = N_c (1 - exp(-nu_ES dt))); with
         * select_mode 1 (Eq. 9 as printed for USP-ESBGK) the N_s =
         * nearest(N_c (1 - exp(-nu_ES dt))) particles with the smallest rank
         * keys are the selected ones */
        double psel = -expm1(-f.x);
        dg[D_PSEL] = psel;
        selinfo* si = (selinfo*)calloc((size_t)nl + 1, sizeof(selinfo));
        const int count_mode = g->scheme != 1 && g->select_mode == 1;
        for (int i = 0; i < nl; ++i) {
            uint32_t r[4];
            draw(g, (uint32_t)o->step, PUR_SELECT, 0, (uint32_t)d, (uint32_t)i, r);
            double u = uspo_uniform(r[0], g->precision);
            si[i].sel = (g->scheme == 1 || count_mode) ? 1 : u < psel;
            double mg = fabs(u - psel);
            if (g->scheme != 1 && !count_mode && mg < dg[D_MARG_SEL]) dg[D_MARG_SEL] = mg;
            si[i].rank = (r[1] & 0xFFFFF800u) | (uint32_t)i;
            si[i].ut = uspo_uniform(r[2], g->precision);
        }
        if (count_mode && nl > 0) {
            /* Eq. 9: nearest integer of N_c (1 - exp(-nu_ES dt)), then the
             * N_s smallest rank keys of the cell */
            const double v = (double)nl * psel;
            int nsel = (int)floor(v + 0.5);
            if (nsel > nl) nsel = nl;
            if (nsel < 0) nsel = 0;
            dg[D_MARG_SEL] = fabs(v - (floor(v) + 0.5));
            uint32_t* all = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)nl);
            for (int i = 0; i < nl; ++i) all[i] = si[i].rank;
            qsort(all, (size_t)nl, sizeof(uint32_t), cmp_rank);
            const uint32_t ths = nsel > 0 ? all[nsel - 1] : 0;
            free(all);
            for (int i = 0; i < nl; ++i) si[i].sel = nsel > 0 && si[i].rank <= ths;
        }
        double S = 0.0;
        int ns = 0;
        for (int i = 0; i < nl; ++i)
            if (si[i].sel) {
                S += L->p[i].w;
                ++ns;
            }
        if (g->scheme == 1) S = (double)ns * psel;
        /* Eq. 28 (Eq. 9 for SP-ESBGK): int() = nearest integer, clamped to
         * [0, N_s] */
        int nusp = (int)floor(S + 0.5);
        dg[D_MARG_ROUND] = fabs(S - (floor(S) + 0.5));
        if (nusp < 0) nusp = 0;
        if (nusp > ns) nusp = ns;
        dg[D_SSEL] = S;
        dg[D_NSEL] = ns;
        dg[D_NUSP] = nusp;
        dg[D_NDEL] = g->scheme == 1 ? 0 : ns - nusp;
        /* keep the nusp selected particles with the smallest rank keys */
        uint32_t* keys = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)ns + 1));
        int j = 0;
        for (int i = 0; i < nl; ++i)
            if (si[i].sel) keys[j++] = si[i].rank;
        qsort(keys, (size_t)ns, sizeof(uint32_t), cmp_rank);
        uint32_t thr = nusp > 0 ? keys[nusp - 1] : 0;
        free(keys);
        for (int i = 0; i < nl; ++i) {
            if (!si[i].sel) si[i].fate = 0;
            else if (nusp > 0 && si[i].rank <= thr) si[i].fate = 1;
            else si[i].fate = g->scheme == 1 ? 0 : 2; /* SP-ESBGK deletes none */
        }

        /* step 6 */
        int nfb = 0;
        for (int i = 0; i < nl; ++i)
            if (si[i].fate == 1) nfb += resample(o, &f, P, d, i, si[i].ut, &L->p[i]);
        dg[D_CHOLFB] = nfb;

        /* step 7 */
        int n7 = spawn(o, 7, d, &f, P, &L7, &dg[D_MARG_CNT]);
        dg[D_N7] = n7;
        if (nl + n7 > g->max_ppc) o->error = -3;

        /* per-cell conservation of mass, momentum and energy */
        if (g->conserve_mode == 0) {
            double Mr = 0, Pr_[3] = {0, 0, 0}, Er = 0;
            for (int pass = 0; pass < 2; ++pass) {
                const part* pp = pass == 0 ? L->p : L7.p;
                int np = pass == 0 ? nl : L7.n;
                for (int i = 0; i < np; ++i) {
                    if (pass == 0 && si[i].fate != 0) continue;
                    double w = pp[i].w;
                    Mr += w;
                    for (int k = 0; k < 3; ++k) Pr_[k] += w * pp[i].c[k];
                    Er += 0.5 * w * (pp[i].c[0] * pp[i].c[0] + pp[i].c[1] * pp[i].c[1] +
                                     pp[i].c[2] * pp[i].c[2]);
                }
            }
            if (nusp == 0) {
                flags |= F_NOUSP;
            } else {
                double Wr = (M0 - Mr) / nusp;
                dg[D_WR] = Wr;
                note_gap(&dg[D_MARG_CONS], Wr, 0.5);
                note_gap(&dg[D_MARG_CONS], Wr, 2.0);
                if (!(Wr >= 0.5 && Wr <= 2.0)) {
                    flags |= F_FAILMASS;
                } else {
                    double MR = Wr * nusp;
                    double a[3], cb[3] = {0, 0, 0};
                    for (int k = 0; k < 3; ++k) a[k] = (P0[k] - Pr_[k]) / MR;
                    for (int i = 0; i < nl; ++i)
                        if (si[i].fate == 1)
                            for (int k = 0; k < 3; ++k) cb[k] += L->p[i].c[k];
                    for (int k = 0; k < 3; ++k) cb[k] /= nusp;
                    double D = 0.0;
                    for (int i = 0; i < nl; ++i)
                        if (si[i].fate == 1)
                            for (int k = 0; k < 3; ++k) {
                                double e = L->p[i].c[k] - cb[k];
                                D += e * e;
                            }
                    double a2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
                    double da2 = 0.0;
                    for (int k = 0; k < 3; ++k) da2 += (a[k] - cb[k]) * (a[k] - cb[k]);
                    double s = 1.0;
                    int shift = 1;
                    if (nusp >= 2 && D > 0.0) {
                        note_gap(&dg[D_MARG_CONS], da2, 9.0 * D / nusp);
                        if (!(da2 <= 9.0 * D / nusp)) {
                            /* the mean would move by more than 3 rms spreads */
                            shift = 0;
                            flags |= F_FAILENERGY;
                        } else {
                            double s2 = (E0 - Er - 0.5 * MR * a2) / (0.5 * Wr * D);
                            dg[D_S2] = s2;
                            note_gap(&dg[D_MARG_CONS], s2, 1.0 / 9.0);
                            note_gap(&dg[D_MARG_CONS], s2, 9.0);
                            if (s2 >= 1.0 / 9.0 && s2 <= 9.0) s = sqrt(s2);
                            else flags |= F_FAILENERGY;
                        }
                    } else {
                        flags |= F_FAILENERGY;
                    }
                    int whole = (flags & F_FAILENERGY) &&
                                whole_cell(o, L, si, nl, &L7, nusp, M0, P0, E0, Mr, Pr_, Er, &dg[D_MARG_CONS]);
                    if (whole)
                        flags = (flags & ~F_FAILENERGY) | F_WHOLE;
                    else
                        for (int i = 0; i < nl; ++i)
                            if (si[i].fate == 1) {
                                part* q = &L->p[i];
                                if (shift)
                                    for (int k = 0; k < 3; ++k)
                                        q->c[k] = st(g, a[k] + s * (q->c[k] - cb[k]));
                                q->w = st(g, Wr);
                            }
                }
                if ((flags & F_FAILMASS) &&
                    whole_cell(o, L, si, nl, &L7, nusp, M0, P0, E0, Mr, Pr_, Er, &dg[D_MARG_CONS]))
                    flags = (flags & ~F_FAILMASS) | F_WHOLE;
            }
        }

        /* compaction: survivors in slot order, then the step-7 particles */
        int w = 0;
        for (int i = 0; i < nl; ++i)
            if (si[i].fate != 2) L->p[w++] = L->p[i];
        L->n = w;
        for (int i = 0; i < L7.n; ++i) pl_push(L, L7.p[i]);
        free(si);
    }
    free(L7.p);
    dg[D_FLAGS] = flags;
    dg[D_NOUT] = L->n;

    /* step 8: moments of f^{n+1} */
    double M1, P1[3], E1;
    totals(L->p, L->n, &M1, P1, &E1);
    dg[D_M1] = M1;
    dg[D_P1X] = P1[0]; dg[D_P1Y] = P1[1]; dg[D_P1Z] = P1[2];
    dg[D_E1] = E1;
    moments(L->p, L->n, o->mom + (size_t)USPO_MOM * d);
    raw_sums(L->p, L->n, o->raw + (size_t)USPO_MOM * d);
}

/* ------------------------------------------------------------------------ */
/* P_ne (Eq. 16-18)                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int valid;
    double rho, T, umag, lam, theta;
} gll_cell;

static void gll_of(const uspo* o, const double m[USPO_MOM], int n, gll_cell* c)
{
    cellf f;
    derive(o, m, n < 0 ? 2 : n, &f);
    c->valid = f.valid;
    if (!f.valid) return;
    c->rho = f.rho;
    c->T = f.T;
    c->theta = f.theta;
    c->umag = sqrt(f.U[0] * f.U[0] + f.U[1] * f.U[1] + f.U[2] * f.U[2]);
    /* Eq. 36 */
    c->lam = 16.0 / (5.0 * sqrt(2.0 * M_PI)) * f.mu / sqrt(f.rho * f.p);
}

/* Kn_GLL,Q = lambda |grad Q| / Q (Eq. 18) for Q = rho, T and |u| (the velocity
 * term scaled by max(|u|, sound speed)); central differences, one-sided next
 * to walls and missing neighbours; P_ne = exp(-max Kn_GLL / Kn_c) (Eq. 16-17). */
static void compute_pne(const uspo* o, const double* mom_centred, const int* counts,
                        double* pout)
{
    const uspo_config* g = &o->g;
    int nc = o->ncell;
    gll_cell* c = (gll_cell*)malloc(sizeof(gll_cell) * (size_t)nc);
    for (int i = 0; i < nc; ++i)
        gll_of(o, mom_centred + (size_t)USPO_MOM * i, counts ? counts[i] : -1, &c[i]);
    for (int i = 0; i < nc; ++i) {
        if (!c[i].valid) {
            pout[i] = 0.0;
            continue;
        }
        int ix = i % g->nx, iy = i / g->nx;
        double g2[3] = {0, 0, 0};
        for (int ax = (g->dim == 2 ? 0 : 1); ax < 2; ++ax) {
            int n = ax == 0 ? g->nx : g->ny;
            int idx = ax == 0 ? ix : iy;
            double h = ax == 0 ? g->dx : g->dy;
            int periodic = g->face_kind[2 * ax] == 2;
            int im = idx - 1, ip = idx + 1;
            if (periodic) {
                im = (im + n) % n;
                ip = ip % n;
            }
            int hm = im >= 0 && im < n, hp = ip >= 0 && ip < n;
            int cm = hm ? (ax == 0 ? iy * g->nx + im : im * g->nx + ix) : -1;
            int cp = hp ? (ax == 0 ? iy * g->nx + ip : ip * g->nx + ix) : -1;
            hm = hm && c[cm].valid;
            hp = hp && c[cp].valid;
            for (int qk = 0; qk < 3; ++qk) {
                double qc = qk == 0 ? c[i].rho : (qk == 1 ? c[i].T : c[i].umag);
                double qm = 0, qp = 0;
                if (hm) qm = qk == 0 ? c[cm].rho : (qk == 1 ? c[cm].T : c[cm].umag);
                if (hp) qp = qk == 0 ? c[cp].rho : (qk == 1 ? c[cp].T : c[cp].umag);
                double gr = 0.0;
                if (hm && hp) gr = (qp - qm) / (2.0 * h);
                else if (hp) gr = (qp - qc) / h;
                else if (hm) gr = (qc - qm) / h;
                g2[qk] += gr * gr;
            }
        }
        double a = sqrt(5.0 / 3.0 * c[i].theta);
        double kr = c[i].lam * sqrt(g2[0]) / c[i].rho;
        double kt = c[i].lam * sqrt(g2[1]) / c[i].T;
        /* Eq. 18 for |u|: over max(|u|, a) or, as printed, over |u| */
        double gu = c[i].lam * sqrt(g2[2]);
        double qu = g->gll_u == 1 ? c[i].umag : (c[i].umag > a ? c[i].umag : a);
        double ku = gu > 0.0 ? (qu > 0.0 ? gu / qu : INFINITY) : 0.0;
        double kn = kr;
        if (kt > kn) kn = kt;
        if (ku > kn) kn = ku;
        pout[i] = exp(-kn / g->Kn_c);
    }
    free(c);
}

static void update_pne(uspo* o, double* pout)
{
    const uspo_config* g = &o->g;
    int nc = o->ncell;
    if (g->pne_mode == 0) {
        for (int i = 0; i < nc; ++i) pout[i] = g->pne_fixed;
        return;
    }
    int* counts = (int*)malloc(sizeof(int) * (size_t)nc);
    for (int i = 0; i < nc; ++i) counts[i] = o->cell[i].n;
    if (g->pne_mode == 2 && (o->n_samples > 0 || g->avg_init)) {
        double* m = (double*)malloc(sizeof(double) * USPO_MOM * (size_t)nc);
        for (int i = 0; i < nc; ++i) {
            centred_from_raw(o->avg + (size_t)USPO_MOM * i, m + (size_t)USPO_MOM * i);
            counts[i] = 2; /* averaged fields: validity from the sums only */
        }
        compute_pne(o, m, counts, pout);
        free(m);
    } else {
        compute_pne(o, o->mom, counts, pout);
    }
    free(counts);
}

/* ------------------------------------------------------------------------ */
/* Lifecycle                                                                 */
/* ------------------------------------------------------------------------ */

static int check_config(const uspo_config* g)
{
    if (g->dim != 1 && g->dim != 2) return -1;
    if (g->nx < 1 || g->ny < 1 || (g->dim == 1 && g->nx != 1)) return -1;
    if (!(g->dt > 0) || !(g->Np > 0) || !(g->vcell > 0) || !(g->r_p > 0)) return -1;
    if (g->precision != 32 && g->precision != 64) return -1;
    if (g->max_ppc < 2 || g->max_ppc > 2048) return -1;
    int open = 0;
    for (int f = 0; f < 4; ++f) {
        if (g->face_kind[f] < 0 || g->face_kind[f] > 3) return -1;
        if (g->face_kind[f] != 3) continue;
        open = 1;
        if (!(g->face_n[f] >= 0.0) || !(g->face_nb[f] >= 0.0)) return -1;
        if (!(g->face_T[f] > 0.0) || !(g->face_Tb[f] > 0.0)) return -1;
        if (g->face_u[3 * f + f / 2] != 0.0) return -1;
    }
    /* a periodic face needs a periodic partner */
    if ((g->face_kind[0] == 2) != (g->face_kind[1] == 2)) return -1;
    if ((g->face_kind[2] == 2) != (g->face_kind[3] == 2)) return -1;
    /* entering particles fly for part of a step: no body force with them */
    if (open && (g->accel[0] != 0.0 || g->accel[1] != 0.0 || g->accel[2] != 0.0)) return -1;
    if (g->plate) {
        if (g->dim != 2 || !(g->plate_x > g->x0 && g->plate_x < g->x1)) return -1;
        if (!(g->plate_ylo <= g->plate_yhi) || !(g->plate_T > 0.0)) return -1;
    }
    /* every mode switch takes one of its listed values */
    if (g->pne_mode < 0 || g->pne_mode > 2) return -1;
    if (g->weight_mode != 0 && g->weight_mode != 1) return -1;
    if (g->conserve_mode != 0 && g->conserve_mode != 1) return -1;
    if (g->jmom_mode != 0 && g->jmom_mode != 1) return -1;
    if (g->spawn_projection != 0 && g->spawn_projection != 1) return -1;
    if (g->avg_init != 0 && g->avg_init != 1) return -1;
    if (g->n_avg < 1) return -1;
    if (g->scheme != 0 && g->scheme != 1) return -1;
    if (g->es_mode != 0 && g->es_mode != 1) return -1;
    if (g->gll_u != 0 && g->gll_u != 1) return -1;
    if (g->select_mode != 0 && g->select_mode != 1) return -1;
    if (g->es_sampler != 0 && g->es_sampler != 1) return -1;
    if (g->es_mode == 1 && !(g->Pr > 0.0 && g->Pr != 1.0)) return -1;
    /* SP-ESBGK has no added particles: P_ne fixed at 0 */
    if (g->scheme == 1 && !(g->pne_mode == 0 && g->pne_fixed == 0.0)) return -1;
    return 0;
}

static uspo* alloc_uspo(const uspo_config* cfg)
{
    if (check_config(cfg)) return NULL;
    uspo* o = (uspo*)calloc(1, sizeof(uspo));
    o->g = *cfg;
    o->ncell = cfg->nx * cfg->ny;
    o->R = cfg->kB / cfg->m;
    o->F = cfg->m * cfg->Np / cfg->vcell;
    size_t nc = (size_t)o->ncell;
    o->cell = (plist*)calloc(nc, sizeof(plist));
    o->mom = (double*)calloc(nc * USPO_MOM, sizeof(double));
    o->raw = (double*)calloc(nc * USPO_MOM, sizeof(double));
    o->avg = (double*)calloc(nc * USPO_MOM, sizeof(double));
    o->avgs = (double*)calloc(nc * USPO_MOM, sizeof(double));
    o->pcur = (double*)calloc(nc, sizeof(double));
    o->pprev = (double*)calloc(nc, sizeof(double));
    o->diag = (double*)calloc(nc * USPO_NDIAG, sizeof(double));
    o->sort_cnt = (int*)calloc(nc, sizeof(int));
    o->sort_perm = NULL;
    o->sort_n = -1;
    return o;
}

static void recompute_cells(uspo* o)
{
    for (int i = 0; i < o->ncell; ++i) {
        moments(o->cell[i].p, o->cell[i].n, o->mom + (size_t)USPO_MOM * i);
        raw_sums(o->cell[i].p, o->cell[i].n, o->raw + (size_t)USPO_MOM * i);
    }
}

/* Table 2 step 1: per cell round(n V / N_p) particles, uniform positions,
 * Maxwellian velocities at the cell's (u, T), weight 1. */
uspo* uspo_create(const uspo_config* cfg, const double* init_n, const double* init_u,
                  const double* init_T)
{
    uspo* o = alloc_uspo(cfg);
    if (!o) return NULL;
    const uspo_config* g = &o->g;
    for (int c = 0; c < o->ncell; ++c) {
        int n = (int)floor(init_n[c] * g->vcell / g->Np + 0.5);
        if (n > g->max_ppc) o->error = -3;
        double sq = sqrt(g->kB * init_T[c] / g->m);
        if (g->avg_init) {
            /* raw sums of a Maxwellian of n particles at (u, theta): sum w = n,
             * sum w c = n u, sum w c c = n (u u + theta I), sum w |c|^2 c =
             * n (|u|^2 + 5 theta) u */
            const double* u = init_u + 3 * c;
            const double th = sq * sq, N = (double)n;
            const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            double* A = o->avgs + (size_t)USPO_MOM * c;
            A[0] = N;
            for (int k = 0; k < 3; ++k) A[1 + k] = N * u[k];
            A[4] = N * (u[0] * u[0] + th);
            A[5] = N * (u[1] * u[1] + th);
            A[6] = N * (u[2] * u[2] + th);
            A[7] = N * u[0] * u[1];
            A[8] = N * u[0] * u[2];
            A[9] = N * u[1] * u[2];
            for (int k = 0; k < 3; ++k) A[10 + k] = N * (u2 + 5.0 * th) * u[k];
            memcpy(o->avg + (size_t)USPO_MOM * c, A, sizeof(double) * USPO_MOM);
        }
        for (int k = 0; k < n; ++k) {
            part q;
            uint32_t r[4];
            draw(g, 0, PUR_INIT_POS, 0, (uint32_t)c, (uint32_t)k, r);
            uniform_position(g, c, r, &q);
            draw(g, 0, PUR_INIT_VEL, 0, (uint32_t)c, (uint32_t)k, r);
            double z[3];
            uspo_normal3(r, g->precision, z);
            for (int d = 0; d < 3; ++d) q.c[d] = st(g, init_u[3 * c + d] + sq * z[d]);
            q.w = 1.0;
            pl_push(&o->cell[c], q);
        }
    }
    recompute_cells(o);
    update_pne(o, o->pcur);
    memcpy(o->pprev, o->pcur, sizeof(double) * (size_t)o->ncell);
    return o;
}

void uspo_destroy(uspo* o)
{
    if (!o) return;
    for (int i = 0; i < o->ncell; ++i) free(o->cell[i].p);
    free(o->cell);
    free(o->mom);
    free(o->raw);
    free(o->avg);
    free(o->avgs);
    free(o->pcur);
    free(o->pprev);
    free(o->diag);
    free(o->sort_cnt);
    free(o->sort_perm);
    free(o);
}

static void one_step(uspo* o)
{
    const uspo_config* g = &o->g;
    int nc = o->ncell;
    memset(o->diag, 0, sizeof(double) * USPO_NDIAG * (size_t)nc);

    /* step 2: particles for f-hat^n, with the moments of f^n and P^{n-1} */
    for (int c = 0; c < nc; ++c) {
        cellf f;
        derive(o, o->mom + (size_t)USPO_MOM * c, o->cell[c].n, &f);
        if (g->jmom_mode == 1 && (o->n_samples > 0 || g->avg_init) && f.valid)
            use_averaged_sh(o, o->avg + (size_t)USPO_MOM * c, &f);
        double mg = INFINITY;
        int n2 = spawn(o, 2, c, &f, o->pprev[c], &o->cell[c], &mg);
        o->diag[(size_t)USPO_NDIAG * c + D_N2] = n2;
        o->diag[(size_t)USPO_NDIAG * c + D_MARG_CNT2] = mg;
        if (o->cell[c].n > g->max_ppc) o->error = -3;
    }

    /* step 3: advection + walls, the particles entering through open faces
     * (after those present, faces in index order), then the stable sort by
     * new cell; particles leaving through open faces are dropped */
    long long total = 0;
    for (int c = 0; c < nc; ++c) o->diag[(size_t)USPO_NDIAG * c + D_MARG_FACE] = INFINITY;
    int* ninj = (int*)calloc((size_t)nc * 4, sizeof(int));
    for (int c = 0; c < nc; ++c) {
        int t = 0;
        for (int f = 0; f < 4; ++f) t += ninj[4 * c + f] = inject_count(g, o->step, c, f);
        if (o->cell[c].n + t > g->max_ppc) o->error = -3;
        o->diag[(size_t)USPO_NDIAG * c + D_NINJ] = t;
        total += o->cell[c].n + t;
    }
    sentry* e = (sentry*)malloc(sizeof(sentry) * (size_t)(total + 1));
    long long k = 0, pre0 = 0;
    int perx = g->face_kind[0] == 2, pery = g->face_kind[2] == 2;
    for (int c = 0; c < nc; ++c) {
        int clamped = 0, gone = 0, n = o->cell[c].n;
        for (int s = 0; s < n + ninj[4 * c] + ninj[4 * c + 1] + ninj[4 * c + 2] + ninj[4 * c + 3];
             ++s) {
            part q;
            int dcell;
            if (s < n) {
                q = o->cell[c].p[s];
                dcell = advect(g, &q, c, s, o->step, &clamped);
            } else {
                int f = 0, j = s - n;
                while (j >= ninj[4 * c + f]) j -= ninj[4 * c + f++];
                dcell = inject_one(g, o->step, c, f, j, s, &q, &clamped);
            }
            if (dcell < 0) {
                ++gone;
                continue;
            }
            note_face_margin(g, o->diag, dcell, &q);
            int sx = c % g->nx, sy = c / g->nx, dx = dcell % g->nx, dy = dcell / g->nx;
            e[k].dest = dcell;
            e[k].dy = min_image(sy - dy, g->ny, pery);
            e[k].dx = min_image(sx - dx, g->nx, perx);
            e[k].slot = s;
            e[k].pre = pre0 + s;
            e[k].q = q;
            ++k;
        }
        pre0 += n + ninj[4 * c] + ninj[4 * c + 1] + ninj[4 * c + 2] + ninj[4 * c + 3];
        o->diag[(size_t)USPO_NDIAG * c + D_CLAMP] = clamped;
        o->diag[(size_t)USPO_NDIAG * c + D_NGONE] = gone;
        o->cell[c].n = 0;
    }
    free(ninj);
    qsort(e, (size_t)k, sizeof(sentry), cmp_entry);
    free(o->sort_perm);
    o->sort_perm = (long long*)malloc(sizeof(long long) * (size_t)(k + 1));
    o->sort_n = k;
    for (int c = 0; c < nc; ++c) o->sort_cnt[c] = 0;
    for (long long i = 0; i < k; ++i) {
        pl_push(&o->cell[e[i].dest], e[i].q);
        o->sort_perm[i] = e[i].pre;
        o->sort_cnt[e[i].dest]++;
    }
    free(e);

    /* steps 4-8 */
    for (int c = 0; c < nc; ++c) relax_cell(o, c, &o->cell[c], o->diag + (size_t)USPO_NDIAG * c);
    /* a moment of f^{n+1} that is not finite poisons the instance (sticky) */
    if (o->error == 0)
        for (size_t i = 0; i < (size_t)nc * USPO_MOM; ++i)
            if (!isfinite(o->raw[i])) {
                o->error = -9;
                break;
            }

    /* Eq. 34 */
    if (o->step >= g->avg_start) {
        double ne = avg_window(g, o->n_samples);
        for (size_t i = 0; i < (size_t)nc * USPO_MOM; ++i)
            o->avg[i] = (ne - 1.0) / ne * o->avg[i] + 1.0 / ne * o->raw[i];
        o->n_samples++;
    }

    /* P_ne for the next step */
    memcpy(o->pprev, o->pcur, sizeof(double) * (size_t)nc);
    update_pne(o, o->pcur);
    o->step++;
}

/* A capacity (-3) or non-finite (-9) error is sticky: the instance takes no
 * further steps (its cells may already hold more particles than the
 * configuration allows, or moments that are not numbers). */
int uspo_step(uspo* o, int nsteps)
{
    for (int i = 0; i < nsteps && o->error == 0; ++i) one_step(o);
    return o->error;
}

int uspo_error(const uspo* o) { return o->error; }

int uspo_ncell(const uspo* o) { return o->ncell; }

long long uspo_num_particles(const uspo* o)
{
    long long t = 0;
    for (int c = 0; c < o->ncell; ++c) t += o->cell[c].n;
    return t;
}

/* parts: [N][6] = x, y, cx, cy, cz, w in canonical order cell by cell;
 * cellstate: [ncell][54] = centred[13], raw[13], avg[13], avg-star[13], P^n, P^{n-1} */
int uspo_get_state(const uspo* o, int* counts, double* parts, double* cellstate, int* step,
                   int* n_samples)
{
    long long k = 0;
    for (int c = 0; c < o->ncell; ++c) {
        if (counts) counts[c] = o->cell[c].n;
        for (int s = 0; s < o->cell[c].n; ++s, ++k) {
            if (!parts) continue;
            const part* q = &o->cell[c].p[s];
            double* r = parts + 6 * k;
            r[0] = q->x; r[1] = q->y; r[2] = q->c[0]; r[3] = q->c[1]; r[4] = q->c[2]; r[5] = q->w;
        }
        if (cellstate) {
            double* cs = cellstate + (size_t)USPO_CS * c;
            memcpy(cs, o->mom + (size_t)USPO_MOM * c, sizeof(double) * USPO_MOM);
            memcpy(cs + USPO_MOM, o->raw + (size_t)USPO_MOM * c, sizeof(double) * USPO_MOM);
            memcpy(cs + 2 * USPO_MOM, o->avg + (size_t)USPO_MOM * c, sizeof(double) * USPO_MOM);
            memcpy(cs + 3 * USPO_MOM, o->avgs + (size_t)USPO_MOM * c, sizeof(double) * USPO_MOM);
            cs[4 * USPO_MOM] = o->pcur[c];
            cs[4 * USPO_MOM + 1] = o->pprev[c];
        }
    }
    if (step) *step = o->step;
    if (n_samples) *n_samples = o->n_samples;
    return 0;
}

/* cellstate may be NULL: moments are then taken from the particles, the
 * averages cleared and P^n = P^{n-1} computed from the instantaneous fields. */
int uspo_set_state(uspo* o, const int* counts, const double* parts, const double* cellstate,
                   int step, int n_samples)
{
    const uspo_config* g = &o->g;
    long long k = 0;
    for (int c = 0; c < o->ncell; ++c) {
        o->cell[c].n = 0;
        for (int s = 0; s < counts[c]; ++s, ++k) {
            const double* r = parts + 6 * k;
            part q;
            q.x = st(g, r[0]); q.y = st(g, r[1]);
            q.c[0] = st(g, r[2]); q.c[1] = st(g, r[3]); q.c[2] = st(g, r[4]);
            q.w = st(g, r[5]);
            pl_push(&o->cell[c], q);
        }
    }
    o->step = step;
    o->n_samples = n_samples;
    o->error = 0;
    o->sort_n = -1;
    if (cellstate) {
        for (int c = 0; c < o->ncell; ++c) {
            const double* cs = cellstate + (size_t)USPO_CS * c;
            memcpy(o->mom + (size_t)USPO_MOM * c, cs, sizeof(double) * USPO_MOM);
            memcpy(o->raw + (size_t)USPO_MOM * c, cs + USPO_MOM, sizeof(double) * USPO_MOM);
            memcpy(o->avg + (size_t)USPO_MOM * c, cs + 2 * USPO_MOM, sizeof(double) * USPO_MOM);
            memcpy(o->avgs + (size_t)USPO_MOM * c, cs + 3 * USPO_MOM, sizeof(double) * USPO_MOM);
            o->pcur[c] = cs[4 * USPO_MOM];
            o->pprev[c] = cs[4 * USPO_MOM + 1];
        }
    } else {
        recompute_cells(o);
        memset(o->avg, 0, sizeof(double) * USPO_MOM * (size_t)o->ncell);
        memset(o->avgs, 0, sizeof(double) * USPO_MOM * (size_t)o->ncell);
        o->n_samples = 0;
        update_pne(o, o->pcur);
        memcpy(o->pprev, o->pcur, sizeof(double) * (size_t)o->ncell);
    }
    return 0;
}

/* Field record per cell (which = 0 instantaneous, 1 averaged):
 * S0, rho, u[3], T, p, sigma[6] (xx yy zz xy xz yz), q[3], P_ne, count. */
int uspo_get_fields(const uspo* o, int which, double* out)
{
    for (int c = 0; c < o->ncell; ++c) {
        double m[USPO_MOM];
        if (which == 1) centred_from_raw(o->avg + (size_t)USPO_MOM * c, m);
        else memcpy(m, o->mom + (size_t)USPO_MOM * c, sizeof(m));
        cellf f;
        derive(o, m, which == 1 ? 2 : o->cell[c].n, &f);
        double* r = out + (size_t)USPO_NF * c;
        memset(r, 0, sizeof(double) * USPO_NF);
        r[0] = m[0];
        r[1] = o->F * m[0];
        for (int k = 0; k < 3; ++k) r[2 + k] = m[1 + k];
        if (f.valid) {
            r[5] = f.T;
            r[6] = f.p;
            for (int k = 0; k < 6; ++k) r[7 + k] = f.p * f.s[k];
            for (int k = 0; k < 3; ++k) r[13 + k] = f.p * f.h[k];
        }
        r[16] = o->pcur[c];
        r[17] = o->cell[c].n;
    }
    return 0;
}

int uspo_get_diag(const uspo* o, double* out)
{
    memcpy(out, o->diag, sizeof(double) * USPO_NDIAG * (size_t)o->ncell);
    return 0;
}

/* The stable counting sort of the last step's step 3 (by new cell; within a
 * cell by source offset, then source slot): counts [ncell] of the sorted
 * particles per cell (the particles of f-tilde^*), perm [N] for each sorted
 * particle its place in the sequence before the sort (cells in order, each
 * with its particles present, then its step-2 particles, then those that
 * entered through open faces; particles that left keep their place).
 * Returns N, or -1 before the first step; either array may be NULL. */
long long uspo_get_sort(const uspo* o, int* counts, long long* perm)
{
    if (o->sort_n < 0) return -1;
    if (counts) memcpy(counts, o->sort_cnt, sizeof(int) * (size_t)o->ncell);
    if (perm && o->sort_n > 0) memcpy(perm, o->sort_perm, sizeof(long long) * (size_t)o->sort_n);
    return o->sort_n;
}

/* ------------------------------------------------------------------------ */
/* Entry points that expose single pieces for the pins                      */
/* ------------------------------------------------------------------------ */

/* Draws one added-particle batch for a cell whose f^n (or f-tilde^*, if
 * starred) has centred moments mom; out = [k][6]. */
int uspo_test_spawn(const uspo_config* cfg, const double mom[USPO_MOM], int n_particles,
                    double pne, int batch, int starred, int cell, int step, double* out,
                    int max_out)
{
    uspo* o = alloc_uspo(cfg);
    if (!o) return -1;
    o->step = step;
    cellf f;
    derive(o, mom, n_particles, &f);
    if (starred && f.valid) {
        double da = 1.0 + cfg->dt * f.nu * pne / 2.0;
        double db = 1.0 + cfg->dt * f.nu * cfg->Pr * pne / 2.0;
        for (int k = 0; k < 6; ++k) f.s[k] /= da;
        for (int k = 0; k < 3; ++k) f.h[k] /= db;
    }
    plist L = {0, 0, 0};
    int n = spawn(o, batch, cell, &f, pne, &L, NULL);
    int m = n < max_out ? n : max_out;
    for (int i = 0; i < m; ++i) {
        double* r = out + 6 * i;
        r[0] = L.p[i].x; r[1] = L.p[i].y;
        r[2] = L.p[i].c[0]; r[3] = L.p[i].c[1]; r[4] = L.p[i].c[2]; r[5] = L.p[i].w;
    }
    free(L.p);
    uspo_destroy(o);
    return n;
}

/* centred moments and field record of a given particle set */
int uspo_test_fields(const uspo_config* cfg, const double* parts, int n, double* out_mom,
                     double* out_fields)
{
    uspo* o = alloc_uspo(cfg);
    if (!o) return -1;
    part* p = (part*)malloc(sizeof(part) * (size_t)(n + 1));
    for (int i = 0; i < n; ++i) {
        const double* r = parts + 6 * i;
        p[i].x = r[0]; p[i].y = r[1];
        p[i].c[0] = r[2]; p[i].c[1] = r[3]; p[i].c[2] = r[4]; p[i].w = r[5];
    }
    double m[USPO_MOM];
    moments(p, n, m);
    if (out_mom) memcpy(out_mom, m, sizeof(m));
    if (out_fields) {
        cellf f;
        derive(o, m, n, &f);
        out_fields[0] = f.valid;
        out_fields[1] = f.rho;
        out_fields[2] = f.T;
        out_fields[3] = f.p;
        for (int k = 0; k < 6; ++k) out_fields[4 + k] = f.p * f.s[k];
        for (int k = 0; k < 3; ++k) out_fields[10 + k] = f.p * f.h[k];
        out_fields[13] = f.nu;
        out_fields[14] = f.mu;
        out_fields[15] = f.valid ? 16.0 / (5.0 * sqrt(2.0 * M_PI)) * f.mu / sqrt(f.rho * f.p) : 0.0;
        out_fields[16] = f.valid ? out_fields[15] / sqrt(8.0 * f.theta / M_PI) : 0.0;
    }
    free(p);
    uspo_destroy(o);
    return 0;
}

/* advects one particle [x, y, cx, cy, cz, w] in place; returns the new cell
 * (-1: it left through an open face) */
int uspo_test_advect(const uspo_config* cfg, double* r, int src_cell, int slot, int step)
{
    part q;
    q.x = r[0]; q.y = r[1]; q.c[0] = r[2]; q.c[1] = r[3]; q.c[2] = r[4]; q.w = r[5];
    int clamped = 0;
    int d = advect(cfg, &q, src_cell, slot, step, &clamped);
    r[0] = q.x; r[1] = q.y; r[2] = q.c[0]; r[3] = q.c[1]; r[4] = q.c[2]; r[5] = q.w;
    return d;
}

/* The particles entering cell c through face `face` at step `step`: up to
 * max_out records (x, y, cx, cy, cz, w, destination cell) into out, the
 * first one at slot `slot0`; a particle that left again has cell -1.
 * Returns the count (-1 for a bad configuration). */
int uspo_test_inject(const uspo_config* cfg, int step, int cell, int face, int slot0,
                     double* out, int max_out)
{
    if (check_config(cfg)) return -1;
    int n = inject_count(cfg, step, cell, face);
    for (int k = 0; k < n && k < max_out; ++k) {
        part q = {0};
        int clamped = 0;
        int d = inject_one(cfg, step, cell, face, k, slot0 + k, &q, &clamped);
        double* r = out + 7 * (size_t)k;
        r[0] = q.x; r[1] = q.y; r[2] = q.c[0]; r[3] = q.c[1]; r[4] = q.c[2]; r[5] = q.w;
        r[6] = d;
    }
    return n;
}

/* P_ne of every cell from given centred moments (validity needs S0 > 0 and a
 * positive trace only) */
int uspo_test_pne(const uspo_config* cfg, const double* mom, double* pne_out)
{
    uspo* o = alloc_uspo(cfg);
    if (!o) return -1;
    compute_pne(o, mom, NULL, pne_out);
    uspo_destroy(o);
    return 0;
}
