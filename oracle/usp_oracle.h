/*
 * CPU oracle of the USP-ESBGK per-time-step particle method
 * (Fei, Zhang, Li, Liu, "A Unified Stochastic Particle Bhatnagar-Gross-Krook
 * Method for Multiscale Gas Flows", arXiv 1808.03801).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, serial, FP64 restatement of the
 * method (Section 3.2, Table 2) used to check the GPU library.  It shares no
 * code with the GPU path.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product never does.
 *
 * Every floating-point computation is done in double precision; particle
 * state is *stored* in the configured precision (float or double) so that the
 * stored numbers are the ones a single-precision solver would hold.
 */
#ifndef USP_ORACLE_H
#define USP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Configuration: plain numbers, filled by the caller. */
typedef struct {
    /* gas: Eq. 35 viscosity law, Pr of Eq. 6 */
    double m, kB, mu_ref, T_ref, omega, Pr;
    /* uniform Cartesian grid; 1-D resolves y only, 2-D resolves x and y */
    int dim, nx, ny;
    double x0, x1, y0, y1, dx, dy, inv_dx, inv_dy, vcell;
    /* faces 0..3 = x-lo, x-hi, y-lo, y-hi; kind 0 diffuse, 1 specular,
     * 2 periodic, 3 open (a reservoir: see face_n below) */
    int face_kind[4];
    double face_T[4];
    double face_u[12];
    double accel[3];
    /* numerics */
    double dt, Np, r_p, Kn_c, pne_fixed;
    int pne_mode, n_avg, avg_start, precision, weight_mode, conserve_mode, max_ppc;
    /* moments that build the added particles and f_G: 0 instantaneous (Eq. 1),
     * 1 time-averaged (Eq. 34); 1 = project each added batch onto zero mass,
     * momentum and energy */
    int jmom_mode, spawn_projection;
    uint32_t seed_lo, seed_hi;
    /* Eq. 34 start: 0 = the first sample, then a running mean until n_avg
     * samples; 1 = the exact raw moments of the initial Maxwellian state,
     * then the fixed window n_avg from the first sample (both averages: the
     * Eq. 34 fields and the averages of f-tilde^*) */
    int avg_init;
    /* open faces (kind 3): the domain touches a reservoir of gas with number
     * density face_n, temperature face_T and velocity face_u (its component
     * normal to the face must be 0).  Where the face's tangential coordinate
     * (x on a y face, y on an x face; 2-D only) is >= face_split, the
     * reservoir has density face_nb and temperature face_Tb instead (a face
     * bordering two chambers). */
    double face_n[4], face_split[4], face_nb[4], face_Tb[4];
    /* internal plate (2-D only): a thin diffuse wall at rest at temperature
     * plate_T on the line x = plate_x, x0 < plate_x < x1, covering
     * plate_ylo <= y <= plate_yhi; both sides reflect */
    int plate;
    double plate_x, plate_ylo, plate_yhi, plate_T;
    /* 0: USP-ESBGK (Table 2); 1: SP-ESBGK (Table 1): no added particles
     * (P_ne fixed at 0), N_s of Eq. 9 particles reassigned, velocities from
     * the fixed target f_G of the cell through the linear map of Eq. 10-11 */
    int scheme;
    /* f_G(t) of step 6: 0 = alpha(t) at a time drawn per particle from
     * Eq. 29-30 (the paper); 1 = its expectation over that time
     * distribution, one Gaussian per cell with the same second moments */
    int es_mode;
    /* velocity term of Eq. 18: 0 = lambda |grad |u|| / max(|u|, sqrt(5 theta
     * / 3)); 1 = lambda |grad |u|| / |u| as printed */
    int gll_u;
    /* step 5 of USP-ESBGK: 0 = each particle selected with probability
     * 1 - exp(-nu_ES dt); 1 = Eq. 9 as printed: N_s = nearest(N_c (1 -
     * exp(-nu_ES dt))) particles, the ones with the smallest rank keys */
    int select_mode;
    /* step 6 sampler of f_G(t): 0 = FP64 Cholesky factor of its covariance;
     * 1 = the linear map of Eq. 10-11 with alpha sigma in place of sigma */
    int es_sampler;
} uspo_config;

/* per-cell state record: centred moments, raw sums, averaged raw sums of f^n,
 * averaged raw sums of f-tilde^*, P_ne^n, P_ne^{n-1} */
#define USPO_MOM 13
#define USPO_CS (4 * USPO_MOM + 2)
/* derived field record (see uspo_get_fields) */
#define USPO_NF 18
/* per-cell diagnostics of the last step */
#define USPO_NDIAG 33

typedef struct uspo uspo;

uspo* uspo_create(const uspo_config* cfg, const double* init_n, const double* init_u,
                  const double* init_T);
void uspo_destroy(uspo* o);
int uspo_step(uspo* o, int nsteps);
int uspo_error(const uspo* o);
long long uspo_num_particles(const uspo* o);
int uspo_ncell(const uspo* o);
int uspo_get_state(const uspo* o, int* counts, double* parts, double* cellstate, int* step,
                   int* n_samples);
int uspo_set_state(uspo* o, const int* counts, const double* parts, const double* cellstate,
                   int step, int n_samples);
int uspo_get_fields(const uspo* o, int which, double* out);
int uspo_get_diag(const uspo* o, double* out);
/* the last step-3 sort: counts [ncell] per cell after it, perm [N] place of
 * each sorted particle in the sequence before it; returns N (-1: no step) */
long long uspo_get_sort(const uspo* o, int* counts, long long* perm);

/* pieces exposed for pinning */
void uspo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double uspo_uniform(uint32_t r, int precision);
void uspo_normal3(const uint32_t r[4], int precision, double z[3]);
double uspo_time_sample(double u, double x, double nu_es, double dt);
int uspo_test_spawn(const uspo_config* cfg, const double mom[USPO_MOM], int n_particles,
                    double pne, int batch, int starred, int cell, int step, double* out,
                    int max_out);
int uspo_test_fields(const uspo_config* cfg, const double* parts, int n, double* out_mom,
                     double* out_fields);
int uspo_test_advect(const uspo_config* cfg, double* part6, int src_cell, int slot, int step);
int uspo_test_inject(const uspo_config* cfg, int step, int cell, int face, int slot0,
                     double* out, int max_out);
int uspo_test_pne(const uspo_config* cfg, const double* mom, double* pne_out);

#ifdef __cplusplus
}
#endif
#endif
