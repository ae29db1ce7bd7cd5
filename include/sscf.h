/* sscf.h -- C ABI of the MI355X (gfx950) sparse SCF library.
 *
 * Method: A. Scemama, N. Renon, M. Rapacioli, "A Sparse SCF algorithm and its
 * parallel implementation: Application to DFTB" (arXiv:1402.2880).
 *
 * The problem (paper, section 2): given the AO overlap S and the reference
 * Kohn-Sham matrix H0 on the atom-neighbour pattern (section 3.2), the DFTB
 * charge term (section 3.7), an initial guess of local MOs (section 3.3) and
 * the sparse threshold eps (section 4.1), iterate the Fock build (step IV) and
 * the partial diagonalization by occupied-virtual rotations (step V, section
 * 3.5), each step followed by re-orthonormalization of the MOs (step III,
 * section 3.4), to self-consistent local MOs, the total energy and the density.
 *
 * Conventions for every call:
 *  - The return value is an sscf_status: SSCF_OK (0) or a negative error code.
 *    sscf_last_error(ctx) gives a human-readable message.  No C++ exception
 *    crosses this interface.
 *  - Array arguments are HOST pointers unless stated otherwise; the library
 *    copies what it needs and never keeps a caller pointer after returning.
 *  - A context is used by one host thread at a time; calls on different
 *    contexts are independent.  All device work of a context runs in order on
 *    the stream given at initialization.
 *  - Every number is FP64 unless stated otherwise; indices are 0-based.
 */
#ifndef SSCF_H
#define SSCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sscf_status;

enum {
  SSCF_OK = 0,
  SSCF_E_INVALID_ARG = -1, /* bad shape, index, pattern, NaN/Inf, NULL pointer      */
  SSCF_E_NOT_SPD = -2,     /* a diagonal element of C^T S C is not positive           */
  SSCF_E_ORTHO = -3,       /* initial orthonormalization did not reach eps/100        */
  SSCF_E_HIP = -4,         /* a HIP runtime call failed (message holds its string)    */
  SSCF_E_STATE = -5,       /* call out of order (e.g. on a failed context)            */
  SSCF_E_CAPACITY = -6,    /* a fixed capacity was exceeded (message names it)        */
  SSCF_E_NOMEM = -7        /* device or host allocation failed                        */
};

enum { SSCF_FP64 = 0, SSCF_FP32_MIXED = 1 };

enum { SSCF_FOCK_H0 = 0, SSCF_FOCK_FULL = 1 };

/* bits of sscf_system_desc.flags */
enum {
  SSCF_FLAG_PROFILE = 1,     /* time the kernel classes with HIP events; count executed matrix-core products */
  SSCF_FLAG_COUNT_WORK = 2   /* count the algorithmic work of each pass (sscf_get_kernel_stats); adds counting
                                kernels and host synchronizations between the passes: for measurement runs */
};

/* Convergence criterion of sscf_control (section 4.1 uses the charge criterion). */
enum { SSCF_CONV_ENERGY = 0, SSCF_CONV_CHARGE = 1 };

/* Thresholds and schedule, changeable between steps (sscf_set_control).  The values
 * at sscf_init_system are eps and e_conv of the descriptor, SSCF_CONV_ENERGY,
 * dq_conv = 0 and step_ortho = 1. */
typedef struct {
  double eps;          /* sparse threshold: H and C cut at eps, Jacobi threshold eps,
                          orthonormalization cut 1e-3 eps and tolerance eps/100 (sec. 4.1) */
  double e_conv;       /* converged when |E(n) - E(n-1)| < e_conv (SSCF_CONV_ENERGY), Ha  */
  double dq_conv;      /* converged when max_a |q_a(n) - q_a(n-1)| < dq_conv (SSCF_CONV_CHARGE) */
  int32_t criterion;   /* SSCF_CONV_ENERGY or SSCF_CONV_CHARGE                           */
  int32_t step_ortho;  /* 1: step III after every step; 0: only at set-up, after
                          convergence (occupied MOs) and on sscf_orthonormalize, the
                          order in which section 2 lists the steps                      */
} sscf_control;

#define SSCF_N_KERNEL_CLASSES 7

typedef struct sscf_ctx sscf_ctx; /* opaque, owned by the library */

/* Optional device allocator (for example a framework's caching allocator).
 * alloc returns device memory of at least `bytes` bytes usable on `stream`, or
 * NULL; free releases it.  When alloc is NULL the library uses hipMalloc/hipFree. */
typedef struct {
  void* self;
  void* (*alloc)(void* self, size_t bytes, void* stream);
  void (*free)(void* self, void* ptr, void* stream);
} sscf_allocator;

/* Problem description.  All arrays are host memory owned by the caller. */
typedef struct {
  /* atoms (section 3.7: minimal valence basis, 1 or 4 AOs per atom) */
  int32_t n_atoms;
  const int32_t* atom_nao;     /* [n_atoms] AOs per atom, 1..4; AOs are numbered atom by atom   */
  const double* xyz_bohr;      /* [n_atoms][3] positions (bohr)                                 */
  const double* hubbard_u;     /* [n_atoms] U (Ha) > 0: gamma_aa = U_a,
                                  gamma_ab = 1/sqrt(r^2 + ((1/U_a + 1/U_b)/2)^2)                */
  const double* q0;            /* [n_atoms] reference valence populations                       */
  const int32_t* atom_group;   /* [n_atoms] MO group of the atom, 0..n_groups-1 (section 3.2)   */
  int32_t n_groups;
  /* atom-neighbour pattern (section 3.2): atom-block CSR, symmetric, self block present,
     columns strictly increasing in each row; block k = (a, blk_col[k]) is the row-major
     atom_nao[a] x atom_nao[b] sub-matrix starting at blk_off[k] of S_val / H0_val */
  const int64_t* blk_rowptr;   /* [n_atoms + 1]                                                 */
  const int32_t* blk_col;      /* [blk_rowptr[n_atoms]]                                          */
  const int64_t* blk_off;      /* [blk_rowptr[n_atoms]]                                          */
  const double* S_val;         /* overlap, symmetric                                            */
  const double* H0_val;        /* reference Kohn-Sham matrix, symmetric (Ha)                    */
  int64_t n_val;               /* length of S_val / H0_val                                      */
  /* molecular orbitals: MO j < n_occ is doubly occupied (closed shell) */
  int32_t n_mo;
  int32_t n_occ;
  const int32_t* mo_group;     /* [n_mo] group of each MO; MOs keep it for the whole SCF        */
  /* initial guess C0 (section 3.3), CSC: column j has rows c0_row[c0_colptr[j] ..
     c0_colptr[j+1]-1], strictly increasing, values c0_val */
  const int64_t* c0_colptr;    /* [n_mo + 1]                                                     */
  const int32_t* c0_row;
  const double* c0_val;
  /* thresholds (section 4.1; section 3.2; section 3.5) */
  double eps;                  /* sparse threshold epsilon, e.g. 1e-5                           */
  double e_conv;               /* SCF converged when |E(n) - E(n-1)| < e_conv (Ha)              */
  double group_nbr_bohr;       /* MO groups are neighbours below this atom-atom distance (20)    */
  double rot_cap_factor;       /* at most rot_cap_factor * n_occ rotations per step (10)        */
  int32_t max_sweeps_init;     /* orthonormalization sweeps allowed at initialization (200)     */
  int32_t max_sweeps_step;     /* orthonormalization sweeps allowed per SCF step (50)           */
  int32_t scc;                 /* 1: add the DFTB charge term of section 3.7; 0: gamma = 0      */
  int32_t precision;           /* SSCF_FP64, or SSCF_FP32_MIXED: C^T H C and the rotation angles
                                  in FP32, everything else in FP64                              */
  void* hip_stream;            /* hipStream_t for all device work; NULL = default stream        */
  sscf_allocator alloc;        /* zero-filled = hipMalloc / hipFree                             */
  uint64_t flags;              /* 0, or SSCF_FLAG_PROFILE | SSCF_FLAG_COUNT_WORK                */
  /* tile capacity of C (section 3.2: the MOs of a group stay near it).  <= 0: every 16-row
     tile of every group has storage (dense capacity, 8 n_groups ceil(n_ao/16) 16 W bytes per
     copy of C: quadratic in the size).  > 0: group g has storage for the row blocks within
     reach_g + slot_margin_bohr of it, reach_g the farthest row block its initial MOs (C0)
     touch; distances between bounding spheres (of the group's atoms, of the block's atoms),
     in bohr.  Memory then grows linearly with the size.  The products Y = X C get the row
     blocks that the pattern of S links to those.  A coefficient of C that would be nonzero
     outside (after the cuts of the method) is an error: SSCF_E_CAPACITY from the call that
     produced it, the context is then failed.  Values the cuts leave zero there are no error. */
  double slot_margin_bohr;
} sscf_system_desc;

/* Per-step report.  Times are device time (HIP events) in milliseconds. */
typedef struct {
  double energy;               /* total energy after the step (Ha)                              */
  double delta_e;              /* energy(n) - energy(n-1)                                       */
  double dq_max;               /* max_a |q_a(n) - q_a(n-1)| (section 4.1)                       */
  double max_abs_fov;          /* largest |F_ia| before the rotations                           */
  double ortho_eta;            /* largest off-diagonal of the normalized C^T S C at exit        */
  double e_band;               /* sum_uv P_uv H0_uv                                             */
  double e_coul;               /* 1/2 sum_ab dq_a gamma_ab dq_b                                 */
  int32_t n_candidates;        /* pairs with |F_ia| >= eps                                      */
  int32_t n_rotations;         /* rotations applied                                             */
  int32_t n_ortho_sweeps;      /* pair-combination sweeps applied                               */
  int32_t converged;           /* |delta_e| < e_conv                                            */
  int32_t ortho_converged;     /* eta < eps/100 was reached                                     */
  int32_t post_ortho;          /* occupied-only orthonormalization was run (once converged)     */
  int64_t nnz_tiles;           /* active 16-row tiles of C                                      */
  int64_t nnz_c;               /* nonzero coefficients of C after the step (with
                                  SSCF_FLAG_COUNT_WORK; -1 without)                             */
  float ms_fock, ms_cfc, ms_select, ms_rot, ms_ortho, ms_sums, ms_total;
} sscf_step_info;

/* Copy the problem to the device, check it, build the neighbour maps and the
 * rotation schedule, and orthonormalize C0 (section 3.4) until the largest
 * off-diagonal of the normalized C^T S C is below eps/100.  On success *out is a
 * new context; on failure *out is NULL and the status tells why
 * (SSCF_E_INVALID_ARG, SSCF_E_NOT_SPD, SSCF_E_ORTHO, SSCF_E_HIP, SSCF_E_NOMEM,
 * SSCF_E_CAPACITY).  The failure message is available from sscf_last_error(NULL). */
sscf_status sscf_init_system(const sscf_system_desc* desc, sscf_ctx** out);

/* Replace the Fock input for the following steps (section 2, step IV).
 * f_val has the layout of S_val (n_val values, host memory).
 * mode SSCF_FOCK_H0:   f_val is a new H0; the charge term is still added each step.
 * mode SSCF_FOCK_FULL: f_val is the complete Fock matrix; no charge term is added
 *                      and the energy becomes sum_uv P_uv F_uv.
 * Errors: SSCF_E_INVALID_ARG (NULL, bad mode, NaN/Inf, not symmetric). */
sscf_status sscf_set_fock(sscf_ctx* ctx, const double* f_val, int32_t mode);

/* Inputs of the GPU initial guess (section 3.3).  A fragment (a molecule) is a run of
 * consecutive atoms; fragments are numbered in atom order. */
typedef struct {
  int32_t n_atoms;
  const int32_t* atom_nao;      /* AOs per atom                                        */
  const int64_t* blk_rowptr;    /* atom-block pattern and values, as in sscf_system_desc */
  const int32_t* blk_col;
  const int64_t* blk_off;
  const double* S_val;
  const double* H0_val;
  int64_t n_val;
  int32_t n_frag;
  const int32_t* atom_frag;     /* fragment of each atom: 0, 0, .., 1, 1, .. (non-decreasing) */
  const int32_t* frag_nocc;     /* doubly occupied MOs of each fragment                */
  const int32_t* frag_group;    /* MO group of each fragment, in [0, n_groups)          */
  int32_t n_groups;
  double drop;                  /* coefficients with |c| < drop are left out of C0       */
  void* hip_stream;             /* stream of the work; NULL = default stream             */
} sscf_guess_desc;

/* Initial guess of section 3.3 on the GPU (one thread per fragment): for every fragment,
 * H0 c = lambda S c restricted to its own AOs (at most 8), solved by Cholesky of S and
 * cyclic Jacobi; each vector's first entry within a relative 1e-10 of its largest |c|
 * is made positive.  C0 is written as CSC
 * into caller-owned host arrays: c0_colptr[n_mo + 1] (n_mo = number of AOs), c0_row[cap],
 * c0_val[cap], mo_group[n_mo].  Column order (the input order of sscf_system_desc): the
 * occupied MOs of group 0, 1, .. (fragments ascending within a group, lambda ascending
 * within a fragment), then the virtual MOs in the same order.  *nnz receives the number of
 * stored coefficients and *n_occ the number of occupied columns, also when cap is too
 * small (then SSCF_E_CAPACITY and nothing else is written).  SSCF_E_INVALID_ARG for
 * inconsistent inputs or a fragment of more than 8 AOs, SSCF_E_NOT_SPD if a fragment's
 * overlap block is not positive definite.  Error text: sscf_last_error(NULL). */
sscf_status sscf_fragment_guess(const sscf_guess_desc* d, int64_t* c0_colptr, int32_t* c0_row, double* c0_val,
                                int64_t cap, int32_t* mo_group, int64_t* nnz, int32_t* n_occ);

/* Atom neighbour map of section 3.2 on the GPU: the atom-block pattern of S and H.  Atoms a
 * and b are neighbours when (dx*dx + dy*dy) + dz*dz < cutoff*cutoff in IEEE double, every
 * operation rounded on its own (two-centre elements vanish beyond their radial cut-off, so
 * every other pair has only zero elements); every atom is its own neighbour.  xyz: n_atoms x 3
 * (host), in the unit of cutoff.  Output in caller-owned host arrays: rowptr[n_atoms + 1],
 * col[cap], the CSR of the map in atom order with ascending columns; the cost grows with the
 * number of 64-atom tiles whose bounding boxes come within the cut-off, so spatially ordered
 * atoms (as the groups of the constrained k-means give) are cheapest.  *nnz receives the number
 * of entries, also when cap is too small or rowptr/col are NULL (then SSCF_E_CAPACITY and
 * nothing else is written).  SSCF_E_INVALID_ARG for n_atoms < 1, a NULL xyz or nnz, a
 * non-finite or |coordinate| > 1e100, or a cutoff outside (0, 1e100].  Error text:
 * sscf_last_error(NULL). */
sscf_status sscf_atom_neighbours(int32_t n_atoms, const double* xyz, double cutoff, void* hip_stream,
                                 int64_t* rowptr, int32_t* col, int64_t cap, int64_t* nnz);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the atom neighbour map of sscf_atom_neighbours with
 * every array in DEVICE memory owned by the caller and no allocation of any kind on the device.
 * xyz: n_atoms x 3 doubles; rowptr: n_atoms + 1 int64, always written; col: cap int32, written
 * when the map fits (col may be NULL to ask for the size).  *nnz (host) receives the number of
 * entries.  The map is the one sscf_atom_neighbours returns, entry for entry.  The call's
 * scratch (tile bounding boxes, per-atom counts, an error flag; about 1.2 MB) is a fixed array
 * that each GPU the library runs on holds until the process ends; every call on a GPU uses that
 * GPU's copy, so calls that overlap on one GPU (from several threads or streams) race: order
 * them.  The call synchronizes the stream twice (to read the size, and before returning, when
 * the scratch is free again).  Errors: SSCF_E_CAPACITY for n_atoms > SSCF_NOALLOC_MAX_ATOMS or
 * cap too small (rowptr and *nnz are then written, col is not); SSCF_E_INVALID_ARG as for
 * sscf_atom_neighbours, or for host pointers.  Error text: sscf_last_error(NULL). */
#define SSCF_NOALLOC_MAX_ATOMS 262144
sscf_status sscf_atom_neighbours_noalloc(int32_t n_atoms, const double* xyz, double cutoff, void* hip_stream,
                                         int64_t* rowptr, int32_t* col, int64_t cap, int64_t* nnz);

/* Inputs of the constrained k-means of section 3.2 (host memory, read during the call). */
typedef struct {
  int32_t n_points;
  const double* points;         /* n_points x 3, row-major (x, y, z of each point)       */
  int32_t n_means;              /* m; m * n_link >= n_points, m <= 4096                   */
  const double* means0;         /* m x 3: starting means (the caller spreads them evenly) */
  int32_t n_link;               /* most points one mean may hold (N_link), <= 1024       */
  int32_t max_iter;             /* iteration cap (>= 1)                                  */
  double tol;                   /* stop once the average displacement of the means < tol */
  void* hip_stream;             /* stream of the work; NULL = a stream of the call's own  */
} sscf_kmeans_desc;

typedef struct {
  int32_t iterations;           /* attribution + move iterations done                    */
  int64_t rounds;               /* parallel proposal rounds, summed over the iterations  */
  double displacement;          /* average displacement of the means in the last one     */
} sscf_kmeans_info;

/* Constrained k-means of section 3.2 on the GPU.  Each iteration links every point to a
 * mean, no mean holding more than n_link points, then moves every mean to the centroid of
 * its points; it stops when the average displacement of the means (sum of |new - old| over
 * the means, divided by m) is below tol, or after max_iter iterations.  The link of each
 * point is the stable attribution: points rank means by increasing squared distance (ties:
 * lower mean index), a full mean keeps its n_link closest points (ties: lower point index),
 * and no point could move to a mean it ranks higher that has room or holds a point ranked
 * below it.  This attribution is unique, so the result does not depend on any visiting
 * order; the section's reshuffling of the means has nothing left to do.  Squared distances are (dx*dx + dy*dy) + dz*dz in IEEE double,
 * rounded operation by operation; centroids are sums in point order divided by the count
 * (an empty mean stays in place).  Outputs (caller-owned host memory): group[n_points] =
 * mean of each point in the last attribution, means[m x 3] = the means after the last
 * move; info may be NULL.  The ordered atom list of the section is the points sorted by
 * (group, index).  SSCF_E_INVALID_ARG for NULL arrays, sizes out of range, m * n_link <
 * n_points, non-finite or |coordinate| > 1e100, max_iter < 1, tol < 0.  The proposal rounds
 * are replayed from a HIP graph captured on the work stream during the call (hence a stream of
 * the call's own when hip_stream is NULL); the call returns after that stream has finished.
 * Error text: sscf_last_error(NULL). */
sscf_status sscf_constrained_kmeans(const sscf_kmeans_desc* d, int32_t* group, double* means,
                                    sscf_kmeans_info* info);

/* Thresholds, criterion and schedule for the following steps (section 4.1; the
 * loose-then-tight run of that section is: loose values, steps until converged,
 * user values, sscf_orthonormalize(ctx, 0, ...), steps).  SSCF_E_INVALID_ARG for
 * negative or non-finite thresholds or unknown criterion / step_ortho values. */
sscf_status sscf_set_control(sscf_ctx* ctx, const sscf_control* c);
sscf_status sscf_get_control(const sscf_ctx* ctx, sscf_control* c);

/* Step III on demand (section 3.4): all MOs (occ_only = 0) or the occupied ones,
 * until eta < eps/100 within the set-up sweep cap, then charges and energy (info
 * may be NULL).  SSCF_E_ORTHO if the cap is reached, SSCF_E_NOT_SPD as at set-up. */
sscf_status sscf_orthonormalize(sscf_ctx* ctx, int32_t occ_only, sscf_step_info* info);

/* One SCF step (section 2, steps IV and V, then step III): Fock build with the
 * charges of the previous step, C^T H C on neighbouring groups, selection and
 * application of the occupied-virtual rotations, re-orthonormalization, Mulliken
 * charges, energy and convergence test; once converged, the occupied MOs are
 * orthonormalized among themselves (section 4.1) and the energy recomputed.
 * `info` may be NULL.  Non-convergence is not an error. */
sscf_status sscf_scf_step(sscf_ctx* ctx, sscf_step_info* info);

/* Total energy (Ha) of the current MOs.  The paper does not write the total energy out; the
 * SCC-DFTB energy of section 3.7 without the repulsive term (a constant here) is used:
 * E = sum_uv P_uv H0_uv + 1/2 sum_ab dq_a gamma_ab dq_b, with dq the Mulliken charges of
 * eq. pop minus q0; after sscf_set_fock(SSCF_FOCK_FULL), E = sum_uv P_uv F_uv. */
sscf_status sscf_get_energy(const sscf_ctx* ctx, double* e_total);

/* Density P = 2 C_occ C_occ^T (section 3.7, eq. pop, closed shell: n_i = 2) on the
 * atom-block pattern of S, written to the caller's host buffer p_val of n_val >= desc.n_val
 * doubles (layout of S_val); the Mulliken charges of eq. pop are sums of P S over it. */
sscf_status sscf_get_density(const sscf_ctx* ctx, double* p_val, size_t n_val);

/* Energy gradient at the current MOs (differentiation form).  The energy of
 * section 3.7 is stationary in the orthonormal occupied MOs at self-consistency,
 * so with the Fock matrix H = H0 + 1/2 S (Q_a + Q_b) of the current charges (not
 * truncated; H = F after sscf_set_fock(SSCF_FOCK_FULL)):
 *   dE_dX = dE/dH0 (dE/dF in complete-Fock mode) = P = 2 C_occ C_occ^T,
 *   dE_dS = dE/dS = -W + 1/2 P (Q_a + Q_b)   (charge term with H0 and SCC only),
 *   W = 2 C_occ (C_occ^T H C_occ) C_occ^T over neighbouring groups (the MOs are
 *   localized, not canonical: the whole occupied-occupied block enters).
 * Each value is the derivative with respect to that stored entry, in the layout of
 * S_val; both are caller-owned host buffers of n_val >= desc.n_val doubles.  The
 * values are derivatives of E once the SCF has converged (|dE| and the
 * occupied-virtual coupling small); before that they are the same expressions at
 * the current MOs.  SSCF_E_INVALID_ARG for NULL buffers or a short n_val. */
sscf_status sscf_get_energy_gradient(sscf_ctx* ctx, double* dE_dX, double* dE_dS, size_t n_val);

/* The same gradient into DEVICE memory of the context's GPU, plus the derivatives with
 * respect to the onsite energies of each atom shell: the onsite energy of a shell sits on
 * the diagonal of H0 (section 3.7), so dE/d(eps_shell) = sum of P_uu over the shell's AOs.
 * dE_dX, dE_dS: n_val >= desc.n_val doubles each (layout of S_val).  dE_donsite: NULL, or
 * n_onsite >= 2 n_atoms doubles: [2a] the atom's s shell (its first AO), [2a + 1] its p shell
 * (its other AOs; 0 for an atom with one AO).  The buffers stay owned by the caller.  The work
 * is enqueued on the context's stream and the call returns without waiting for it: the
 * values are ready for later work on that stream, or after synchronizing it.  Nothing is
 * copied to or from the host.  SSCF_E_INVALID_ARG for NULL or host buffers or short sizes. */
sscf_status sscf_get_energy_gradient_device(sscf_ctx* ctx, double* dE_dX, double* dE_dS, size_t n_val,
                                            double* dE_donsite, size_t n_onsite);

/* Device memory the context holds now (bytes, its own allocations), the tile slots of each
 * pool of C and of each pool of the products Y = X C (see slot_margin_bohr), and the number
 * of (group, 16-row block) tiles.  All pointers must be non-NULL (else SSCF_E_INVALID_ARG). */
sscf_status sscf_memory_info(const sscf_ctx* ctx, size_t* device_bytes, int64_t* tile_slots, int64_t* tile_slots_y,
                             int64_t* tiles);

/* Mulliken populations q_a (section 3.7, eq. pop) into q[n_atoms] (host). */
sscf_status sscf_get_charges(const sscf_ctx* ctx, double* q, size_t n);

/* The MOs as CSC (rows increasing).  Call with row == NULL to get *nnz; then
 * with arrays colptr[n_mo + 1], row[*nnz], val[*nnz] (host).  Entries are the
 * nonzero coefficients. */
sscf_status sscf_get_mo_coefficients(const sscf_ctx* ctx, int64_t* colptr, int32_t* row,
                                     double* val, int64_t* nnz);

/* The report of the initialization (orthonormalization sweeps, eta, energy). */
sscf_status sscf_init_info(const sscf_ctx* ctx, sscf_step_info* info);

/* Jacobi blocks (occupied group g, virtual group h) and their rounds, in the
 * order they are applied: g[n], h[n], round[n] with n = *n_blocks.  Call with
 * g == NULL to get *n_blocks. */
sscf_status sscf_get_schedule(const sscf_ctx* ctx, int32_t* g, int32_t* h, int32_t* round,
                              int32_t* n_blocks);

/* The rotations (section 3.5) the last step selected and applied, as (occupied MO, virtual MO)
 * pairs in the order of application within each Jacobi block (decreasing |F_ia|), block by
 * block in the order of sscf_get_schedule: occ[k], virt[k] for k < *n.  Call with occ == NULL
 * to get *n (0 before the first step); with arrays, *n gives their room (SSCF_E_INVALID_ARG if
 * too small).  Host arrays, caller-owned. */
sscf_status sscf_get_rotations(const sscf_ctx* ctx, int32_t* occ, int32_t* virt, int64_t* n);

/* Work and time of the main kernel classes, accumulated over the steps, set-up and step III
 * calls since initialization (or the last reset).  Classes: spmm_tiles (the products Y = X C:
 * H C of C^T H C, S C of each orthonormalization sweep, H0 C_occ of the band energy),
 * pair_overlap (C^T S C over neighbouring groups, section 3.4), pair_fock (occupied-virtual
 * C^T H C of the Jacobi blocks, section 3.5), ortho_update (the pair combinations C - 1/2 C D_sel,
 * section 3.4, with the packing of C's nonzero columns it reads), rotations (composition of each
 * Jacobi block's rotations and the pass over the row blocks, section 3.5, with the recount of
 * the tile flags after the cut), select, fock.
 *  launches, ms: with SSCF_FLAG_PROFILE, the launches of the class and their summed HIP-event time.
 *  mfma_flops:   with SSCF_FLAG_PROFILE, 2048 flops per executed 16 x 16 x 4 matrix-core product
 *                of the class (zero operands and padding included: the tiled execution).
 *  alg_flops, alg_bytes: with SSCF_FLAG_COUNT_WORK (else -1), the algorithmic work of the
 *                class, counted on the library's state at each pass; nnz counts nonzero values,
 *                a flop is one multiplication or addition of the sparse operation itself, each
 *                nonzero FP64 value read or written counts 8 bytes (4 in FP32), once:
 *     spmm_tiles:   2 sum_{nu, j} [C_nu,j != 0] nnz(X row nu);  8 (nnz X + nnz C + nnz Y)
 *     pair_overlap: 2 sum |supp C_i ∩ supp (S C)_j| over each unordered pair of MOs of
 *                   neighbouring groups once (i of the lower group; i <= j inside a group);
 *                   8 (nnz C + nnz S C + pairs)
 *     pair_fock:    the same over the occupied i and virtual a of the Jacobi blocks
 *     ortho_update: 2 sum_{(i, j) selected, i != j} nnz C_i;  8 (nnz C before + selected
 *                   pairs + nnz C after)
 *     rotations:    6 n_rot(b) |U(b)| per Jacobi block b, U(b) the rows where one of the block's
 *                   columns is nonzero when the block starts; 16 bytes per nonzero of those columns
 *   The same definitions, counted by the test oracle on its own state, pin these counts.
 * Call with out == NULL to get *n. */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;                   /* summed HIP-event time of the launches                         */
  double mfma_flops;
  double alg_flops;
  double alg_bytes;
} sscf_kernel_stat;

sscf_status sscf_get_kernel_stats(const sscf_ctx* ctx, sscf_kernel_stat* out, int32_t* n);
sscf_status sscf_reset_kernel_stats(sscf_ctx* ctx);

/* Release the context and all its device memory. */
void sscf_destroy(sscf_ctx* ctx);

/* Last error message of ctx (or of the last failed sscf_init_system if ctx is NULL). */
const char* sscf_last_error(const sscf_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
