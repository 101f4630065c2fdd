/*
 * cmc.h -- C ABI of the Coulomb-process Monte Carlo library (libcmc.so).
 *
 * Implements, for MI355X (gfx950), the per-cell pairwise Monte Carlo step
 * of Martinez et al., "High-Energy Radiation and Pair Production by Coulomb
 * Processes in Particle-In-Cell Simulations" (Sec. III.A): weighted
 * macro-electrons and macro-photons are paired with the macro-ions of their
 * cell and undergo Bremsstrahlung (Sec. II.B), Bethe-Heitler (Sec. II.C)
 * and Coulomb Trident (Sec. II.D) events, with cross sections screened by
 * the Thomas-Fermi-Debye potential (Sec. II.A, eq:V_TFD).  A deterministic
 * expected-yield pass and its adjoint sit beside the step.
 *
 * Conventions shared by every entry point
 *  - Units: momenta in m_e c (photons: k times the unit direction), energies
 *    in m_e c^2, densities in m^-3, temperatures in eV, times in s, cross
 *    sections in m^2.  Weights are in density units: the density of a
 *    species in a cell is the sum of its weights (Sec. III.A).
 *  - Pointers named "device" are device memory owned by the caller; the
 *    library keeps no reference to them after the call returns.  Host
 *    pointers are read before the call returns.
 *  - Calls enqueue work on `stream` (a hipStream_t passed as void*, NULL =
 *    the default stream) and return without synchronising.
 *  - Argument errors found on the host return CMC_EINVAL (or CMC_ERANGE)
 *    synchronously, enqueue nothing and set the thread-local message of
 *    cmc_last_error().  Among them: a device array whose address is not a
 *    multiple of its element size (8 for double and int64, 4 for int32).  Errors found on the device (bad cell parameters,
 *    bad weights, energies above the tables, full product buffers, cells
 *    larger than the launch allows) never abort the launch: they set bits
 *    of the sticky status word (CMC_ST_*) and are counted in the tallies.
 *  - No call allocates device memory except cmc_build_tables.
 */
#ifndef CMC_H
#define CMC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CMC_OK = 0,
    CMC_EINVAL = 1,    /* bad argument (null or misaligned pointer, size,   */
                       /* flag)                                             */
    CMC_ERANGE = 2,    /* argument outside the supported range              */
    CMC_EDEVICE = 3,   /* HIP runtime error (launch, copy, memory)          */
    CMC_ENOMEM = 4     /* device allocation failed (cmc_build_tables only)  */
} cmc_status;

/* Thread-local text of the last error reported by this thread. */
const char* cmc_last_error(void);

/* processes (bit mask), Sec. II.B, II.C, II.D */
enum { CMC_BREMS = 1, CMC_BH = 2, CMC_TRIDENT = 4 };
/* arithmetic of the table lookups and kinematics; the event probability
 * 1 - exp(-x) and all tallies are FP64 in both forms */
enum { CMC_FP64 = 0, CMC_FP32 = 1 };

/* sticky device status bits */
enum {
    CMC_ST_OVERFLOW = 1,    /* a product buffer of some cell was full       */
    CMC_ST_GAMMA_HIGH = 2,  /* an energy above the table top (clamped)      */
    CMC_ST_BAD_CELL = 4,    /* Z* outside [0, Z], n_i <= 0 or T < 0: skipped */
    CMC_ST_BAD_WEIGHT = 8,  /* a negative or non-finite weight: cell skipped */
    CMC_ST_TOO_LARGE = 16,  /* a cell above max_per_cell: cell skipped       */
    CMC_ST_BAD_OFFSETS = 32 /* expected yield: a cell's offsets decrease or
                               leave [0, n_part]: cell skipped               */
};

/* ------------------------------------------------------------------ */
/* Cross-section tables (Sec. III.A: cross sections tabulated in the   */
/* ion rest frame)                                                      */
/* ------------------------------------------------------------------ */
typedef struct cmc_tables_s* cmc_tables;

/* Build all tables for element Z (1..100) on the current device: total
 * Bremsstrahlung cross section and its photon-energy moment, Bethe-Heitler
 * total cross section, and the cumulative distributions used to sample
 * photon, pair and positron energies (numerical inversion of the
 * cumulative distribution, Sec. III.A), for the screened potential of
 * eq:V_TFD (non-relativistic segment, eq:cs_br_nr) and its reduced
 * single-exponential form (eq:csre, eq:csur, eq:dsdkbh).  The grid is fixed
 * (see the package documentation); FP64 and FP32 copies are kept.
 * Allocates device memory (about 45 MB) and enqueues the build on `stream`;
 * the handle is usable by any later work ordered after it.
 * Errors: CMC_EINVAL (Z out of range, out == NULL), CMC_ENOMEM, CMC_EDEVICE. */
cmc_status cmc_build_tables(int32_t Z, void* stream, cmc_tables* out);

/* Free the tables (synchronises the device first).  NULL is a no-op. */
cmc_status cmc_tables_free(cmc_tables t);

/* Number of FP64 values of table array `which` (0..12, in the order
 * sigR, skR, cdfR, sigU, skU, cdfU, sigN, skN, cdfN, sigB, cdfB, cdfT, cdfS),
 * or -1 if `which` is unknown. */
int64_t cmc_tables_size(cmc_tables t, int32_t which);

/* Copy table array `which` (FP64) to host memory `dst` of n values
 * (synchronous).  Errors: CMC_EINVAL (bad handle, which, n), CMC_EDEVICE. */
cmc_status cmc_tables_export(cmc_tables t, int32_t which, double* dst, int64_t n);

/* ------------------------------------------------------------------ */
/* Particle layout: structure of arrays, grouped by cell.  Cell c owns   */
/* positions [off[c], off[c+1]) of every array of the species; the first */
/* count[c] of them are live (count == NULL: all of them).  The others   */
/* hold no particle: a step may leave any value there.                   */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n_cells;
    const double* Zstar;   /* device [n_cells]: ionisation degree, 0 <= Z* <= Z */
    const double* n_i;     /* device [n_cells]: ion density for screening (eq:LDH) */
    const double* T_e;     /* device [n_cells]: temperature T_e = T_i, eV */
    const int64_t* cell_id;/* device [n_cells]: global index of each cell, the
                              cell word of every Philox counter (only its low
                              32 bits are used); NULL = the position c.  With
                              global indices a subset of the cells, or the
                              cells split over several launches, draws the
                              same numbers as one launch over all of them */
} cmc_cells;

typedef struct {
    const int64_t* off;    /* device [n_cells+1], non-decreasing             */
    int32_t* count;        /* device [n_cells] live counts, or NULL (= full)  */
    double *px, *py, *pz;  /* device momenta, m_e c (photons: k n).  Ions:
                              proper velocity u = gamma_i beta_i, all three
                              set, or all NULL for ions at rest            */
    double* w;             /* device weights                                  */
    int64_t* parent;       /* device, products only (NULL = not recorded):
                              global index of the parent particle            */
} cmc_species;

typedef struct {
    double dt;             /* time step, s (> 0)                              */
    uint64_t seed;         /* Philox key                                      */
    uint64_t step;         /* step counter (keys the random numbers)          */
    uint32_t processes;    /* CMC_BREMS | CMC_BH | CMC_TRIDENT                */
    int32_t precision;     /* CMC_FP64 or CMC_FP32                            */
    int32_t schedule;      /* 0 = automatic, see CMC_SCHED_*                  */
    int32_t max_per_cell;  /* upper bound of live electrons, photons and ions
                              per cell (<= CMC_MAX_PER_CELL); sizes the launch */
    double near_rel;       /* band |U - P| <= near_rel * P counted as near-threshold,
                              in [0, 1] (default 1e-6)                        */
    void* pass_events[2];  /* optional hipEvent_t pair (both or none), to time
                              the pair-test kernels of the step: [0] is
                              stamped by the first of them at its start, [1]
                              recorded on the stream after the last (no
                              marker between kernels); ignored by
                              CMC_SCHED_CELL                                  */
    uint64_t* step_counter;/* optional device [1] (NULL: use `step`): the step
                              number is read from it on the device and it is
                              incremented by the step, so that a step captured
                              in a HIP graph runs the next step on each replay */
} cmc_step_params;

#define CMC_MAX_PER_CELL 16384

/* per-cell tallies: int64 [n_cells][CMC_NI] and FP64 [n_cells][CMC_ND] */
enum { CMC_I_PAIRS_BR = 0, CMC_I_PAIRS_TR, CMC_I_PAIRS_BH,
       CMC_I_EV_BR, CMC_I_EV_TR, CMC_I_EV_BH,
       CMC_I_NEAR_BR, CMC_I_NEAR_TR, CMC_I_NEAR_BH,
       CMC_I_DROP_PH, CMC_I_DROP_EL, CMC_I_DROP_PO, CMC_NI };
enum { CMC_D_NAB_EI = 0,   /* n_ei = sum_j min(W_e, W_i), eq:proba3          */
       CMC_D_NAB_GI,       /* same for photon-ion pairs                      */
       CMC_D_E_BR,         /* sum W k of Bremsstrahlung photons              */
       CMC_D_E_TR,         /* sum W (g+ + g-) of Trident pairs               */
       CMC_D_E_BH,         /* sum W (g+ + g-) of Bethe-Heitler pairs         */
       CMC_D_DE_EL,        /* sum W (gamma_after - gamma_before), electrons,
                              from the ion-frame loss dE' = -k / -g_pair:
                              gamma_i dE' + u.n' (|p'_f| - |p'|), which is
                              dE' for ions at rest                          */
       CMC_D_DE_PH,        /* -sum W k of photons converted                  */
       CMC_D_W_BR, CMC_D_W_TR, CMC_D_W_BH,  /* created weight per process    */
       CMC_ND };

typedef struct {
    int64_t* ti;           /* device [n_cells*CMC_NI], overwritten            */
    double* td;            /* device [n_cells*CMC_ND], overwritten            */
    int32_t* status;       /* device [1], OR-ed with CMC_ST_* (caller clears) */
} cmc_tallies;

/* ------------------------------------------------------------------ */
/* Pairing (Sec. III.A): in every cell, N = max(N_a, N_b) macro-pairs,   */
/* each drawn uniformly.  Each species is put in a random order by a     */
/* 32-bit Philox4x32-10 key per particle (ties broken by index); the     */
/* larger species A is walked once in that order and the smaller B       */
/* cyclically: pair j = (A[pi_A(j)], B[pi_B(j mod N_B)]); on a tie the   */
/* a-species is A.  pass = 1 keys electrons/ions as the electron-ion     */
/* pass of cmc_collide_step does, pass = 2 photons/ions.                 */
/* a_off/b_off/pair_off: device [n_cells+1]; a_cnt/b_cnt device or NULL; */
/* wa/wb device weights; pair_off[c] = caller's exclusive scan of        */
/* max(N_a, N_b).  Outputs (device): pa[pair_off[c]+j], pb[...] = local  */
/* index (within the cell) of the a and b particle of pair j; n_ab       */
/* (nullable) [n_cells] = sum_j min(W_a, W_b).                           */
/* cell_id: device [n_cells] global cell indices keying the draws, or   */
/* NULL = position (as in cmc_cells).                                    */
/* Cells with more than CMC_MAX_PER_CELL particles of a species produce  */
/* no pairs and set pa = pb = -1.                                        */
/* Errors: CMC_EINVAL (null pointers, pass), CMC_EDEVICE.                */
/* ------------------------------------------------------------------ */
cmc_status cmc_pair_cells(int64_t n_cells, const int64_t* cell_id, const int64_t* a_off, const int32_t* a_cnt,
                          const int64_t* b_off, const int32_t* b_cnt,
                          const double* wa, const double* wb,
                          uint64_t seed, uint64_t step, uint32_t pass,
                          const int64_t* pair_off, int32_t* pa, int32_t* pb, double* n_ab,
                          void* stream);

/* ------------------------------------------------------------------ */
/* One Monte Carlo step (Sec. III.A, eq:proba3), all cells.             */
/*  1. electron-ion pass: per pair, Bremsstrahlung then Trident on the   */
/*     electron as left by Bremsstrahlung;                               */
/*  2. photon-ion pass: Bethe-Heitler over the photons live at the start */
/*     of the step.                                                      */
/* Each pair: P = 1 - exp(-(n_a n_b/n_ab) sigma' gamma' v'/(gamma_a      */
/* gamma_b) dt) in FP64; the event happens iff U1 < P and               */
/* U2 < W_ion/max(W_mobile, W_ion); the energy is sampled from the      */
/* tabulated cumulative distribution; products move along the parent.   */
/* Primed quantities are in the rest frame of the pair's ion, reached   */
/* by the boost along the ion velocity (Sec. III.A; the photon's flux   */
/* factor is k' c/(k gamma_i)); products are boosted back to the lab.   */
/* With ions at rest (ion px = py = pz = NULL) the frames coincide.     */
/* Updates in place: electron momenta; photons (Bremsstrahlung photons   */
/* are appended to the photon species of the cell, photons converted by  */
/* Bethe-Heitler are removed and the survivors kept in order, followed   */
/* by the new photons; photons->count is required).  Trident and        */
/* Bethe-Heitler e- and e+ are appended to new_el / new_po (count       */
/* required, capacity off[c+1]-off[c]); products are appended in pair    */
/* order; a full buffer drops the product (counted, CMC_ST_OVERFLOW).    */
/* Random numbers: Philox4x32-10 keyed by (seed) with counter            */
/* (pair or particle index, cell, step, tag), the cell word taken from   */
/* cells->cell_id: results do not depend on the schedule, and with       */
/* global cell indices not on how cells are split across launches or    */
/* devices (without cell_id each launch numbers its cells from 0).       */
/* workspace: device scratch of cmc_step_workspace_bytes() bytes (may be */
/* NULL when that is 0).                                                 */
/* Errors: CMC_EINVAL (null or inconsistent pointers, dt <= 0, unknown  */
/* processes/precision/schedule, near_rel outside [0, 1], ion momenta  */
/* neither all set nor all NULL), CMC_ERANGE                             */
/* (max_per_cell outside [1, CMC_MAX_PER_CELL]), CMC_EDEVICE.            */
/* ------------------------------------------------------------------ */
cmc_status cmc_collide_step(cmc_tables t, const cmc_cells* cells,
                            cmc_species* electrons, cmc_species* photons,
                            const cmc_species* ions,
                            cmc_species* new_el, cmc_species* new_po,
                            const cmc_step_params* params, cmc_tallies* tallies,
                            void* workspace, size_t workspace_bytes, void* stream);

/* Scratch bytes cmc_collide_step needs for n_cells with this schedule. */
size_t cmc_step_workspace_bytes(int64_t n_cells, int32_t schedule);

/* ------------------------------------------------------------------ */
/* For callers that cannot allocate device memory (code under HIP graph */
/* capture, tight serving loops, harnesses that forbid hipMalloc): the  */
/* step of cmc_collide_step with no workspace argument.  Its scratch is */
/* a file-scope device array of the library, one per GPU it runs on,    */
/* sized for cmc_noalloc_max_cells() cells (16384, about 10 MB) and     */
/* held until the process ends.  Every call on a GPU shares that GPU's  */
/* array, which keeps the last call's contents (each step clears what   */
/* it needs before use): calls that overlap on one GPU race.  The call  */
/* allocates nothing; an automatic schedule never times team shapes     */
/* here (it takes the shape an earlier cmc_collide_step chose for the   */
/* same launch shape, else workgroup teams).  Results are those of      */
/* cmc_collide_step.  Errors: as cmc_collide_step, and CMC_ERANGE for   */
/* more cells than the array holds.                                      */
/* ------------------------------------------------------------------ */
cmc_status cmc_collide_step_noalloc(cmc_tables t, const cmc_cells* cells,
                                    cmc_species* electrons, cmc_species* photons,
                                    const cmc_species* ions,
                                    cmc_species* new_el, cmc_species* new_po,
                                    const cmc_step_params* params, cmc_tallies* tallies,
                                    void* stream);

/* Cells cmc_collide_step_noalloc's static workspace holds. */
size_t cmc_noalloc_max_cells(void);

/* Schedules (every schedule gives the same decisions and products):
 *  CMC_SCHED_CELL   one workgroup per cell tests the pairs in order (the
 *                   sequential reference schedule; no workspace);
 *  CMC_SCHED_GROUP  all pairs of a cell are tested at once from the state
 *                   at the start of the step by one workgroup per cell,
 *                   events are then applied in pair order; cells where a
 *                   particle used by a later pair changes (or with many
 *                   events, or too many particles for LDS) fall back to
 *                   the sequential kernel;
 *  CMC_SCHED_WAVE   the same with one wavefront per cell (cells above
 *                   1024 particles of a species take the fallback);
 *  CMC_SCHED_HYBRID wavefronts for the cells with at most 1024 particles of
 *                   every species, workgroups for the larger ones (uneven
 *                   cells);
 *  CMC_SCHED_QUEUE  workgroups that take the cells from a work queue, in
 *                   decreasing order of cost (pairs of both passes): one
 *                   workgroup per entry, dispatched in queue order as
 *                   compute units free up, so the costliest cells start
 *                   first (the batched form for uneven cells);
 *  CMC_SCHED_SPLIT  workgroups for the electron-ion pass, then one
 *                   wavefront per cell for the photon-ion pass (its order,
 *                   when it needs one, of up to 256 photons; larger orders
 *                   take a workgroup): for a few photons cycled against
 *                   many ions, as in a foil's Bremsstrahlung -> Bethe-
 *                   Heitler chain;
 *  CMC_SCHED_AUTO   GROUP, WAVE (max_per_cell <= 1024) or HYBRID, QUEUE
 *                   and, with both passes on, SPLIT, each with and without
 *                   the stream kernel, whichever is fastest on the first
 *                   step of a
 *                   launch shape (device, n_cells, max_per_cell, processes,
 *                   precision): that first call times them and waits for
 *                   the timing; under stream capture an untimed shape uses
 *                   GROUP. */
enum { CMC_SCHED_AUTO = 0, CMC_SCHED_CELL = 1, CMC_SCHED_GROUP = 2, CMC_SCHED_WAVE = 3, CMC_SCHED_HYBRID = 4,
       CMC_SCHED_QUEUE = 5, CMC_SCHED_SPLIT = 6 };
/* Every schedule but CELL and WAVE first runs the stream kernel: one
 * workgroup walks each cell whose ions are at rest and whose electrons
 * each pair once (N_i <= N_e, 1024 < N_e <= 4096), reading every record
 * once for both passes; the other cells take the schedule's teams.  OR-ing
 * CMC_SCHED_NO_STREAM into the schedule leaves every cell to its teams (the
 * same decisions and products). */
#define CMC_SCHED_NO_STREAM 0x100

/* ------------------------------------------------------------------ */
/* Expected photon energy yield (deterministic): for every cell c,      */
/*   Y_c = sum_j w_j P_j <k>_j,  P = 1 - exp(-n_i sigma_B(gamma) beta c dt), */
/* each electron against the cell's ions at rest with n_i = n_e/Z*      */
/* (eq:proba1, eq:LDH), <k> = sigma_k/sigma_B the mean photon energy of */
/* the tabulated spectrum.  Zstar, n_e, T_e: device [n_cells]; off      */
/* device [n_cells+1]; px..w device [n_part] (n_part >= off[n_cells]);  */
/* Y device [n_cells]; y_part device [n_part] per-electron terms or     */
/* NULL; status device [1] or NULL, OR-ed with CMC_ST_* (caller clears).*/
/* precision: CMC_FP64 or CMC_FP32 (table lookups in FP32, P and sums   */
/* in FP64).  A cell without electrons gets Y = 0.  Checked per cell on */
/* the device: a cell whose offsets decrease or leave [0, n_part] is    */
/* skipped (Y = 0, nothing else written; CMC_ST_BAD_OFFSETS), and a cell */
/* with Z* outside (0, Z], n_e <= 0 or T_e < 0 (or a non-finite value)  */
/* gets Y = 0 and zero terms (CMC_ST_BAD_CELL).  n_cells = 0 does       */
/* nothing, and then every array may be NULL.                           */
/* Errors: CMC_EINVAL (NULL arrays, dt <= 0, n_part < 0, precision),    */
/* CMC_EDEVICE.                                                         */
/* ------------------------------------------------------------------ */
cmc_status cmc_expected_yield(cmc_tables t, int64_t n_cells, const double* Zstar,
                              const double* n_e, const double* T_e, const int64_t* off,
                              int64_t n_part, const double* px, const double* py, const double* pz,
                              const double* w, double dt, int32_t precision,
                              double* Y, double* y_part, int32_t* status, void* stream);

/* Adjoint of cmc_expected_yield for upstream gradient gY (device
 * [n_cells]): writes dL/dpx, dL/dpy, dL/dpz, dL/dw (per electron, device
 * [n_part]; gw may be NULL) and dL/dZ*, dL/dn_e, dL/dT_e (per cell),
 * L = sum_c gY_c Y_c.  The table lookups are recomputed, not stored.  The
 * derivative of the piecewise-linear table interpolant is taken inside the
 * bracketing interval (one-sided at knots), the interval being located
 * from the FP64 energy in both forms.  A cell without electrons gets zero
 * cell gradients.  Cells are checked as in cmc_expected_yield: a cell with
 * bad offsets is skipped (zero cell gradients, CMC_ST_BAD_OFFSETS), a bad
 * cell gets zero gradients (CMC_ST_BAD_CELL).  n_cells = 0 does nothing,
 * and then every array may be NULL.  Errors: CMC_EINVAL, CMC_EDEVICE. */
cmc_status cmc_expected_yield_backward(cmc_tables t, int64_t n_cells, const double* Zstar,
                                       const double* n_e, const double* T_e, const int64_t* off,
                                       int64_t n_part, const double* px, const double* py,
                                       const double* pz, const double* w, double dt,
                                       int32_t precision, const double* gY, double* gpx,
                                       double* gpy, double* gpz, double* gw, double* gZstar,
                                       double* gn_e, double* gT_e, int32_t* status, void* stream);

/* ------------------------------------------------------------------ */
/* Screening forms (Sec. II.B.2).  The cross sections of the           */
/* relativistic regimes (eq:csre, eq:csur) and of Bethe-Heitler pair   */
/* production (eq:dsdkbh) see the atomic potential through the         */
/* screening functions I1, I2 (eq:defphi1, eq:defphi2).  The step uses */
/* the reduced potential, one exponential of length L_R (eq:reduit,    */
/* eq:lambert-W), whose functions have closed forms (eq:deriv_I1,      */
/* eq:deriv_I2).  These calls give them in either form: the reduced    */
/* one, or that of the two-exponential Thomas-Fermi-Debye potential    */
/* itself (eq:V_TFD), computed by quadrature -- the comparison of      */
/* Figs. 5, 7 and 8.                                                    */
/* ------------------------------------------------------------------ */
enum { CMC_SCREEN_REDUCED = 0, CMC_SCREEN_TFD = 1 };

/* I1[i], I2[i] at delta[i] (eq:defphi1, eq:defphi2) for the cell state  */
/* (Zstar[i], n_i[i], T_e[i]) of point i (Sec. II.A, for the element of */
/* the tables t) in screening form `form`.  Every array is a device     */
/* array of n doubles owned by the caller; status is a device int32 or  */
/* NULL, OR-ed with CMC_ST_* (caller clears).  A point with delta       */
/* outside (0, 1] or an invalid cell state (Z* outside [0, Z], n_i <= 0, */
/* T_e < 0 or non-finite) gets NaN in both outputs and sets              */
/* CMC_ST_BAD_CELL.  n = 0 does nothing (the arrays may then be NULL).  */
/* Asynchronous on stream.  Errors: CMC_EINVAL (NULL handle or array,   */
/* unknown form, n < 0), CMC_EDEVICE.                                   */
cmc_status cmc_screening_functions(cmc_tables t, int32_t form, int64_t n, const double* Zstar,
                                   const double* n_i, const double* T_e, const double* delta,
                                   double* I1, double* I2, int32_t* status, void* stream);

/* Differential cross sections at n points in screening form `form`,     */
/* each with its cell state as above:                                    */
/*   process CMC_BREMS: e1[i] = gamma_1 >= 2, x[i] = k/(gamma_1 - 1) in  */
/*     (0, 1); out[i] = k dsigma/dk in m^2, eq:csre for gamma_1 <= 100   */
/*     and eq:csur (Coulomb correction f_C(Z)) above;                    */
/*   process CMC_BH: e1[i] = k > 2, x[i] = (gamma_+ - 1)/(k - 2) in      */
/*     (0, 1); out[i] = dsigma/dgamma_+ in m^2, eq:dsdkbh.               */
/* Device arrays of n doubles, caller-owned; an invalid point gets NaN   */
/* and sets CMC_ST_BAD_CELL.  Errors as for cmc_screening_functions, and */
/* CMC_EINVAL for another process.                                       */
cmc_status cmc_cross_sections(cmc_tables t, int32_t process, int32_t form, int64_t n,
                              const double* Zstar, const double* n_i, const double* T_e,
                              const double* e1, const double* x, double* out, int32_t* status,
                              void* stream);

/* ------------------------------------------------------------------ */
/* The step after.  Created particles are macro-particles of their      */
/* species (Sec. III.A): the photons one step creates convert in the    */
/* next (a step appends them to the photon population itself), and the  */
/* electrons and positrons of a pair radiate and make pairs in turn (the */
/* chains of Sec. IV).  These calls move particle records on the device; */
/* species as for cmc_collide_step, device pointers, caller-owned, all   */
/* asynchronous on stream.                                               */
/* ------------------------------------------------------------------ */
/* Cell by cell, appends the live particles of src after the live ones   */
/* of dst, in src's order, as far as dst's slab of the cell holds them;  */
/* sets dst->count, and src->count to 0.  Particles that do not fit are  */
/* dropped: their number per cell goes to dropped (device [n_cells], or  */
/* NULL) and CMC_ST_OVERFLOW is OR-ed into *status (device, or NULL).    */
/* Both species need count, off and w; px, py, pz on both or neither;    */
/* parent is copied when both have it.  n_cells = 0 does nothing.        */
/* Errors: CMC_EINVAL (NULL arrays, missing counts), CMC_EDEVICE.        */
cmc_status cmc_merge_species(int64_t n_cells, const cmc_species* dst, const cmc_species* src,
                             int64_t* dropped, int32_t* status, void* stream);

/* New slabs for a species: off_new (device [n_cells+1]) gets           */
/* off_new[0] = 0, off_new[c+1] = off_new[c] + live(c) + headroom,        */
/* live(c) the cell's live count (count == NULL: its whole slab).  The   */
/* caller reads off_new[n_cells], allocates the new arrays and calls     */
/* cmc_rebin_copy.  Errors: CMC_EINVAL (NULL, n_cells < 0, headroom < 0), */
/* CMC_EDEVICE.                                                          */
cmc_status cmc_rebin_offsets(int64_t n_cells, const cmc_species* src, int32_t headroom,
                             int64_t* off_new, void* stream);

/* Copies each cell's live particles of src to the start of its slab in  */
/* dst (dst->off from cmc_rebin_offsets) and sets dst->count to their    */
/* number; the rest of each slab is left as it is.  Arrays as for        */
/* cmc_merge_species (dst->count required).  Errors: CMC_EINVAL,         */
/* CMC_EDEVICE.                                                          */
cmc_status cmc_rebin_copy(int64_t n_cells, const cmc_species* src, const cmc_species* dst, void* stream);

#ifdef __cplusplus
}
#endif
#endif
