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

/* ---- measurement only: nothing below changes a result ------------------------------ */

/* Algorithmic work of the passes of one step, counted on the oracle's own state at the
 * point where each pass runs (counting on: orc_set_count).  "nnz" counts stored values
 * that are not zero; a flop is one multiplication or addition of the sparse operation
 * itself, never of a padded or tiled form of it; bytes count each nonzero FP64 value read
 * or written once (8 bytes).
 *  ORC_W_PRODUCT:  Y = X C on the MOs of the pass (X = H for C^T H C, S in every sweep
 *                  of step III, H0 on the occupied MOs for the band energy sum_i C_i^T H0 C_i):
 *                  flops 2 sum_{nu, j} [C_nu,j != 0] nnz(X row nu); bytes 8 (nnz X + nnz C + nnz Y)
 *  ORC_W_OVERLAP:  C^T S C over neighbouring groups, each unordered MO pair once, i from
 *                  the lower group (lower local index within a group):
 *                  flops 2 sum |supp C_i ∩ supp Y_j|; bytes 8 (nnz C + nnz Y + pairs)
 *  ORC_W_FOCK_BLOCKS: occupied-virtual C_i^T (H C)_a of the Jacobi blocks, same counts
 *  ORC_W_COMBINE:  C <- C - 1/2 C D_sel: flops 2 sum_{(i, j) selected, i != j} nnz C_i;
 *                  bytes 8 (nnz C before + nnz C after + selected pairs)
 *  ORC_W_ROTATE:   per Jacobi block, its rotations over the union U_b of the rows of its
 *                  columns at the block's start: flops 6 n_rot_b |U_b|; bytes 16 times the
 *                  nonzeros of those columns at the block's start (read and written once) */
enum { ORC_W_PRODUCT = 0, ORC_W_OVERLAP = 1, ORC_W_FOCK_BLOCKS = 2, ORC_W_COMBINE = 3, ORC_W_ROTATE = 4,
       ORC_W_N = 5 };
#define ORC_W_MAX_SWEEPS 64
typedef struct {
  double flops[ORC_W_N];
  double bytes[ORC_W_N];
  int32_t passes[ORC_W_N];
  int32_t n_sweeps;                          /* combination sweeps of the call           */
  int64_t sweep_sel[ORC_W_MAX_SWEEPS];       /* selected ordered pairs (i, j), i != j     */
  int64_t sweep_nnz_in[ORC_W_MAX_SWEEPS];    /* nnz of C (MOs of the sweep) entering      */
  int64_t sweep_nnz_out[ORC_W_MAX_SWEEPS];   /* and leaving the combination               */
  double sweep_flops[ORC_W_MAX_SWEEPS];
} orc_work;

/* counting on (1) or off (0, the default); the counts cover the last orc_step, set-up or
 * orc_orthonormalize call made with counting on */
int orc_set_count(orc_t* o, int32_t on);
int orc_work_get(const orc_t* o, orc_work* out);

/* Trace of the combination sweeps of the last call (on: orc_set_trace; for small systems):
 * for sweep k, C entering the combination (normalized; CSC over the sweep's MOs) and the
 * selected ordered pairs (i, j) with their D_ij, in the order the sweep visits them. */
int orc_set_trace(orc_t* o, int32_t on);
int orc_trace_sweeps(const orc_t* o);
int orc_trace_sizes(const orc_t* o, int32_t k, int32_t* n_scope, int64_t* nnz, int64_t* n_sel, double* eta);
int orc_trace_get(const orc_t* o, int32_t k, int64_t* colptr, int32_t* row, double* val, int32_t* sel_i,
                  int32_t* sel_j, double* sel_d);

/* last step's occupied-virtual C^T H C blocks, concatenated in block order, each row-major
 * (occupied MOs of g) x (virtual MOs of h); *n receives the length (call with out NULL) */
int orc_fov(const orc_t* o, double* out, int64_t* n);
/* the truncated Fock matrix of the last step on the atom-block pattern (layout of S_val) */
int orc_fock(const orc_t* o, double* out);

#ifdef __cplusplus
}
#endif
#endif
