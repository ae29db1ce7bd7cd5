/* FP64 CPU oracle of the sparse SCF hot path (Scemama, Renon, Rapacioli,
 * "A Sparse SCF algorithm and its parallel implementation: Application to DFTB").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that the
 * HIP library is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header, table
 * or helper with the HIP library.
 *
 * Every reduction is done per output element in a fixed order, so results do
 * not depend on the number of OpenMP threads.
 */
#ifndef SSCF_ORACLE_H
#define SSCF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc orc_t;

typedef struct {
  int32_t n_atoms;
  const int32_t* atom_nao;      /* AOs per atom (1 or 4)                       */
  const double* xyz_bohr;       /* [n_atoms][3]                                 */
  const double* hubbard_u;      /* Ha                                           */
  const double* q0;             /* reference valence populations                */
  const int32_t* atom_group;    /* MO group of the atom's molecule              */
  int32_t n_groups;
  const int64_t* blk_rowptr;    /* atom-block CSR pattern, self block included  */
  const int32_t* blk_col;
  const int64_t* blk_off;       /* offset of the row-major nao_a x nao_b block  */
  const double* S_val;
  const double* H0_val;
  int32_t n_mo;
  int32_t n_occ;                /* MOs 0..n_occ-1 are doubly occupied           */
  const int32_t* mo_group;
  const int64_t* c0_colptr;     /* initial guess, CSC, rows sorted per column   */
  const int32_t* c0_row;
  const double* c0_val;
  double eps;                   /* sparse threshold epsilon                     */
  double e_conv;                /* |dE| convergence threshold (Ha)              */
  double r_nbr_bohr;            /* MO-group neighbour distance (20 bohr)        */
  double rot_cap_factor;        /* at most factor * n_occ rotations per step    */
  int32_t max_sweeps_init;      /* orthonormalization sweeps at set-up          */
  int32_t max_sweeps_step;      /* orthonormalization sweeps per SCF step       */
  int32_t scc;                  /* 1: DFTB charge term; 0: gamma = 0            */
  int32_t n_threads;            /* 0: OpenMP default                            */
} orc_desc;

typedef struct {
  double energy;                /* total energy after the step (Ha)             */
  double delta_e;
  double dq_max;                /* max_a |q_a(n) - q_a(n-1)|                    */
  double max_abs_fov;           /* max |F_ia| before the rotations              */
  double ortho_eta;             /* last max off-diagonal of normalized C^T S C  */
  double e_band, e_coul;
  int32_t n_candidates;         /* |F_ia| >= threshold                          */
  int32_t n_rotations;
  int32_t n_ortho_sweeps;       /* combination sweeps applied                   */
  int32_t converged;
  int32_t ortho_converged;
  int32_t post_ortho;           /* occupied-only orthonormalization was run     */
  int64_t nnz_c;
  double t_fock, t_fmo, t_select, t_rotate, t_ortho, t_charges, t_energy; /* s */
} orc_step_info;

int orc_create(const orc_desc* d, orc_t** out);
void orc_destroy(orc_t* o);
const char* orc_last_error(const orc_t* o);

/* one SCF step: Fock build, C^T H C, rotation selection and application,
 * re-orthonormalization, charges, energy; occupied-only orthonormalization
 * once converged */
int orc_step(orc_t* o, orc_step_info* info);

/* replace the Fock matrix for the next step (values on the atom-block pattern):
 * mode 0: new H0 (charge term still added); mode 1: complete Fock, no charge term */
int orc_set_fock(orc_t* o, const double* f_val, int32_t mode);

/* thresholds and schedule from the next step on (section 4.1): sparse threshold eps;
 * convergence criterion 0 = |dE| < e_conv, 1 = dq_max < dq_conv (the paper's);
 * step_ortho 1 = step III after every step, 0 = only at set-up and after convergence
 * (the order in which section 2 lists the steps) */
int orc_set_control(orc_t* o, double eps, double e_conv, double dq_conv, int32_t criterion, int32_t step_ortho);
/* The paper's literal variants, for quantifying the readings (not for parity):
 * literal_rot: truncation |C| < eps after every single rotation instead of after each block;
 * literal_ortho: the selected pairs combined one at a time in ascending (i, j) order, each
 * pair's columns cut at 1e-3 eps at once, instead of C <- C - 1/2 C D_sel. */
int orc_set_literal(orc_t* o, int32_t literal_rot, int32_t literal_ortho);

/* step III on demand: all MOs (only_occ = 0) or the occupied ones; then charges, energy */
int orc_orthonormalize(orc_t* o, int32_t only_occ, orc_step_info* info);

/* set-up summary: orthonormalization sweeps, final eta, energy */
int orc_init_info(const orc_t* o, orc_step_info* info);

double orc_energy(const orc_t* o);
/* P = 2 C_occ C_occ^T on the atom-block pattern (same layout as S_val) */
int orc_density(const orc_t* o, double* p_val);
int orc_charges(const orc_t* o, double* q);
/* C as CSC; colptr[n_mo+1]; returns -1 if cap is too small */
int64_t orc_nnz_c(const orc_t* o);
int orc_get_c(const orc_t* o, int64_t* colptr, int32_t* row, double* val, int64_t cap);

/* Jacobi block schedule: n_blocks, then per block (g, h, round) */
int orc_n_blocks(const orc_t* o);
int orc_schedule(const orc_t* o, int32_t* g, int32_t* h, int32_t* round);
/* group neighbour map, n_groups x n_groups bytes */
int orc_group_nbr(const orc_t* o, uint8_t* out);

/* last step's F (diagonal over all MOs) and rotation list (i, a, c, s) */
int orc_fdiag(const orc_t* o, double* out);
int orc_n_rot(const orc_t* o);
int orc_rotations(const orc_t* o, int32_t* i, int32_t* a, double* c, double* s);

/* energy gradient at the current MOs (atom-block pattern, layout of S_val):
 * dx = dE/dH0 (dE/dF with a complete Fock matrix), ds = dE/dS */
int orc_gradient(orc_t* o, double* dx_val, double* ds_val);

/* the 2x2 rotation of one (occupied i, virtual a) pair from F_ii, F_aa, F_ia */
void orc_jacobi_angle(double fii, double faa, double fia, double* c, double* s);

#ifdef __cplusplus
}
#endif
#endif
