/*
 * cmc_oracle.h -- interface of the FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the HIP path is checked against.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the HIP library: every formula here is written out
 * again from the paper (Martinez et al., "High-Energy Radiation and Pair
 * Production by Coulomb Processes in Particle-In-Cell Simulations").
 *
 * Units: momenta in m_e c, energies in m_e c^2, cross sections in m^2,
 * densities in m^-3, temperatures in eV, times in s.  Weights are in
 * density units, so that the density of a species in a cell is the sum of
 * its weights (Sec. III.A).
 */
#ifndef CMC_ORACLE_H
#define CMC_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* processes (bit mask) */
#define OR_BREMS   1u
#define OR_BH      2u
#define OR_TRIDENT 4u

/* per-cell integer tallies, [n_cells][OR_NI] */
enum { OR_I_PAIRS_BR = 0, OR_I_PAIRS_TR, OR_I_PAIRS_BH,
       OR_I_EV_BR, OR_I_EV_TR, OR_I_EV_BH,
       OR_I_NEAR_BR, OR_I_NEAR_TR, OR_I_NEAR_BH,
       OR_I_DROP_PH, OR_I_DROP_EL, OR_I_DROP_PO,
       OR_NI };
/* per-cell FP64 tallies, [n_cells][OR_ND] */
enum { OR_D_NAB_EI = 0, OR_D_NAB_GI,
       OR_D_E_BR,      /* sum W k of Bremsstrahlung photons (lab)        */
       OR_D_E_TR,      /* sum W (g+ + g-) of Trident pairs (lab)         */
       OR_D_E_BH,      /* sum W (g+ + g-) of Bethe-Heitler pairs (lab)   */
       OR_D_DE_EL,     /* sum W (gamma_after - gamma_before), electrons,
                          from the energy given to the products       */
       OR_D_DE_PH,     /* sum W (-k) of photons converted by BH          */
       OR_D_W_BR, OR_D_W_TR, OR_D_W_BH,   /* created weight per process  */
       OR_ND };
/* sticky status bits */
#define OR_ST_OVERFLOW   1
#define OR_ST_GAMMA_HIGH 2
#define OR_ST_BAD_CELL   4
#define OR_ST_BAD_WEIGHT 8

typedef struct or_tables_s or_tables;

typedef struct {
    int64_t n_cells;
    const double* Zstar;   /* ionization degree per cell, in [0, Z] */
    const double* n_i;     /* ion density for screening, m^-3       */
    const double* T_e;     /* temperature, eV                        */
    const int64_t* cell_id;/* global cell index keying Philox, NULL = position */
} or_cells;

typedef struct {
    const int64_t* off;    /* [n_cells+1] segment bounds              */
    int32_t* count;        /* [n_cells] live count, NULL = full       */
    double *px, *py, *pz;  /* momenta (photons: k n), ions: u = g*beta or NULL */
    double* w;             /* weights                                 */
    int64_t* parent;       /* products only: global parent index      */
} or_species;

/* table build for element Z (1..100); returns 0 on success */
int  or_tables_build(int Z, or_tables** out);
void or_tables_free(or_tables* t);
/* size / export of one table array, see oracle.py for the names */
int64_t or_tables_size(const or_tables* t, int which);
int  or_tables_export(const or_tables* t, int which, double* dst, int64_t n);

/* physics entry points used by the pins */
void   or_gauss_legendre(int n, double* x, double* w);
double or_lambert_w0(double z);
double or_fc(double Z);
void   or_I12(double delta, double L, double* I1, double* I2);
double or_I_tfd(double etf, double ed, double Ltf, double Ld);
void   or_I12_tfd(double delta, double etf, double ed, double Ltf, double Ld, double* I1, double* I2);
double or_dsdk_rel_tfd(double Z, double g1, double k, double etf, double ed, double Ltf, double Ld, int coulomb);
double or_dsdgp_bh_tfd(double Z, double k, double gp, double etf, double ed, double Ltf, double Ld);
double or_L_reduced(double a);
void   or_screening(double Z, double Zs, double ni, double T, double out[8]);
double or_dsdk_nr(double Z, double g1, double k, double etd, double Ltf, double Ld, int elwert);
double or_dsdk_rel(double Z, double g1, double k, double L, int coulomb);
double or_dsdgp_bh(double Z, double k, double gp, double L);
double or_sigma_trident(double Z, double g1);
double or_dsdgp_trident(double Z, double g1, double gpair);
double or_split_shape(double gpair, double gplus);
void   or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_u53(uint32_t a, uint32_t b);
/* U1 and U2 of the acceptance test of the pair keyed by x (see the .c file) */
void or_accept_uniforms(uint64_t seed, uint64_t step, uint32_t cell, uint32_t x, uint32_t tag,
                        uint32_t tag_hi, double* U1, double* U2);
/* Sec. III.A boost to / from the rest frame of an ion of proper velocity
 * u = gamma_i beta_i: out = (E', p') and p (momentum only) */
void   or_to_ion(const double u[3], double E, const double p[3], double out[4]);
void   or_from_ion(const double u[3], double Ep, const double pp[3], double out[3]);

/* cross sections looked up from the tables for one cell state */
int or_lookup(const or_tables* t, double Zs, double ni, double T, double gamma_or_k,
              int process, double out[4]);
/* inverse-CDF sample from the tables: returns the sampled energy(s) */
int or_sample(const or_tables* t, double Zs, double ni, double T, double e1,
              int process, double xi1, double xi2, double out[2]);

/* cell_id: global cell index keying Philox (NULL = position) */
int or_pair_cells(int64_t n_cells, const int64_t* cell_id, const int64_t* a_off, const int32_t* a_cnt,
                  const int64_t* b_off, const int32_t* b_cnt,
                  const double* wa, const double* wb,
                  uint64_t seed, uint64_t step, uint32_t pass,
                  const int64_t* pair_off, int32_t* pa, int32_t* pb, double* n_ab);

int or_collide_step(const or_tables* t, const or_cells* cells,
                    or_species* el, or_species* ph, const or_species* ion,
                    or_species* new_el, or_species* new_po,
                    double dt, uint64_t seed, uint64_t step, uint32_t processes,
                    double near_rel, int64_t* tal_i, double* tal_d, int32_t* status,
                    int nthreads);

int or_expected_yield(const or_tables* t, int64_t n_cells, const double* Zs,
                      const double* n_e, const double* T_e, const int64_t* off,
                      const double* px, const double* py, const double* pz,
                      const double* w, double dt, double* Y, double* y_part, int nthreads);

int or_expected_yield_backward(const or_tables* t, int64_t n_cells, const double* Zs,
                      const double* n_e, const double* T_e, const int64_t* off,
                      const double* px, const double* py, const double* pz,
                      const double* w, double dt, const double* gY,
                      double* gpx, double* gpy, double* gpz, double* gw,
                      double* gZs, double* gne, double* gTe,
                      double* gabs /* [n_cells][3] sum of |terms| of each cell gradient, or NULL */,
                      int nthreads);

/* The step after: append src to dst cell by cell (dropped per cell, may be
 * NULL; src emptied), and new slabs with headroom for a species. */
void or_merge_species(int64_t n_cells, or_species* dst, or_species* src, int64_t* dropped);
void or_rebin_offsets(int64_t n_cells, const or_species* s, int32_t headroom, int64_t* off_new);
void or_rebin_copy(int64_t n_cells, const or_species* s, or_species* d);

#ifdef __cplusplus
}
#endif
#endif
