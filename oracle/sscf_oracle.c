/* FP64 CPU oracle of the sparse SCF hot path.
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow reference the HIP library is
 * checked against.  Only the tests, the smoke check and the CPU baseline leg of
 * the benchmark load it.  It shares no code with the HIP library.
 *
 * Paper: A. Scemama, N. Renon, M. Rapacioli, "A Sparse SCF algorithm and its
 * parallel implementation: Application to DFTB" (arXiv:1402.2880).
 *
 * Data structures are deliberately simple: S, H0 and H as an AO-level CSR
 * matrix, C as one sorted sparse column per MO (the list-of-lists idea of
 * section 3.1, without padding), C^T S C and the occupied-virtual block of
 * C^T H C as dense blocks per pair of neighbouring MO groups (section 3.2:
 * blocks between non-neighbouring groups are taken as zero).
 *
 * Readings of points the paper leaves open (each one also applied by the HIP
 * library):
 *  - orthonormalization (section 3.4): every sweep recomputes C^T S C,
 *    normalizes with its diagonal, tests the largest off-diagonal of the
 *    normalized matrix D against eps/100, and otherwise applies the pair
 *    combinations of all pairs with |D_ij| >= 1e-3 * max|D| simultaneously,
 *    C <- C - 1/2 C D_sel, then zeroes |C_ki| < 1e-3 eps in the combined
 *    columns (section 4.1);
 *  - partial diagonalization (section 3.5): the rotation of the pair (i, a)
 *    uses the angle from the F of the start of the step; the second rotation
 *    formula is read as C'_a = -s C_i + c C_a (the printed one is not a
 *    rotation); sgn(0) = +1; candidates are |F_ia| >= eps, at most
 *    rot_cap_factor * n_occ of them, the largest first (ties by (i, a));
 *    they are applied block round by block round (figure of the C^T H C
 *    blocks), inside a block by decreasing |F_ia|; after each block the
 *    rotated columns lose their |C_ki| < eps entries (section 4.1);
 *  - DFTB (section 3.7): gamma_aa = U_a, gamma_ab = 1/sqrt(r^2 + u^2) with
 *    u = (1/U_a + 1/U_b)/2, r in bohr; |H_uv| < eps is set to zero;
 *    E = sum_uv P_uv H0_uv + 1/2 sum_ab dq_a gamma_ab dq_b with
 *    P = 2 C_occ C_occ^T (closed shell);
 *  - each SCF step ends with a full re-orthonormalization; once |dE| < e_conv
 *    the occupied MOs are orthonormalized among themselves (section 4.1) and
 *    the charges and energy recomputed.
 *
 * A literal mode (orc_set_literal, not used for parity) takes the two
 * order-dependent steps as the sections print them: truncation after every
 * single rotation, and the pairs combined one at a time in ascending (i, j)
 * order, each from the columns as they stand.  It measures how far the two
 * readings above move the converged energy.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_NOT_SPD = -2, ORC_E_ORTHO = -3, ORC_E_ALLOC = -4 };

typedef struct {
  int32_t n;
  int32_t* row;
  double* val;
} col_t;

struct orc {
  double eps, e_conv, r_nbr, rot_cap_factor;
  double dq_conv;       /* dq_max criterion (section 4.1)                           */
  int criterion;        /* 0: |dE| < e_conv; 1: dq_max < dq_conv                     */
  int step_ortho;       /* 1: step III after every step; 0: at set-up and after convergence */
  int max_sweeps_init, max_sweeps_step, scc, fock_full;
  int literal_rot, literal_ortho;   /* the paper's literal variants (quantification only) */
  int n_atoms, n_ao, n_mo, n_occ, n_groups;
  int32_t* atom_nao;
  int64_t* ao_off;
  int32_t* ao_atom;
  double *xyz, *U, *q0;
  int32_t* atom_group;
  int64_t* blk_rowptr;
  int32_t* blk_col;
  int64_t* blk_off;
  int64_t nblk, nblkval;
  /* AO-level CSR of S / H0 / H */
  int64_t* rp;
  int32_t* ci;
  int64_t* ao2blk;
  double *S, *H0, *H, *Fuser;
  /* MOs */
  int32_t* mo_group;
  int32_t* mo_local;
  col_t* C;
  int32_t *gm_ptr, *gm, *g_nocc;
  uint8_t* gnbr;
  int32_t *gn_ptr, *gn, *gn_pos;
  /* C^T S C blocks for ordered neighbour pairs (g, k-th neighbour of g) */
  int64_t* ob_off;
  double* O;
  /* Jacobi blocks */
  int n_blocks, n_rounds;
  int32_t *jb_g, *jb_h, *jb_round, *jb_of;
  int64_t* jb_foff;
  double *F, *Fdiag;
  /* last step's rotations */
  int n_rot;
  int32_t *rot_i, *rot_a, *rot_blk;
  double *rot_c, *rot_s;
  /* state */
  double *q, *q_prev, *dq, *Q, *P;
  double E, e_band, e_coul;
  orc_step_info init_info;
  char err[256];
  /* measurement only (orc_set_count, orc_set_trace) */
  int count_on, trace_on;
  orc_work work;
  int n_trace, cap_trace;
  struct trace_sweep* trace;
};

struct trace_sweep {
  int32_t n_scope;
  int64_t nnz, n_sel;
  double eta;
  int64_t* colptr;
  int32_t *row, *si, *sj;
  double *val, *sd;
};

/* ----------------------------------------------------------------------------------- */

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* Neumaier's compensated sum */
typedef struct { double s, c; } ksum_t;
static void ks_add(ksum_t* k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
  else k->c += (x - t) + k->s;
  k->s = t;
}
static double ks_get(const ksum_t* k) { return k->s + k->c; }

static int fail(orc_t* o, int code, const char* msg) {
  snprintf(o->err, sizeof(o->err), "%s", msg);
  return code;
}

static void* xcalloc(size_t n, size_t sz) {
  if (n == 0) n = 1;
  return calloc(n, sz);
}

static void col_free(col_t* c) {
  free(c->row);
  free(c->val);
  c->row = NULL;
  c->val = NULL;
  c->n = 0;
}

static double col_dot_dense(const col_t* c, const double* y) {
  double s = 0.0;
  for (int32_t t = 0; t < c->n; ++t) s += c->val[t] * y[c->row[t]];
  return s;
}

/* y = X c for a symmetric AO matrix X (CSR); touched rows are appended to list */
static int32_t spmv_col(const orc_t* o, const double* X, const col_t* c, double* y,
                        uint8_t* mark, int32_t* list) {
  int32_t nt = 0;
  for (int32_t t = 0; t < c->n; ++t) {
    const int32_t nu = c->row[t];
    const double cv = c->val[t];
    for (int64_t k = o->rp[nu]; k < o->rp[nu + 1]; ++k) {
      const int32_t mu = o->ci[k];
      if (!mark[mu]) { mark[mu] = 1; list[nt++] = mu; }
      y[mu] += X[k] * cv;
    }
  }
  return nt;
}

static void clear_touched(double* y, uint8_t* mark, const int32_t* list, int32_t nt) {
  for (int32_t t = 0; t < nt; ++t) { y[list[t]] = 0.0; mark[list[t]] = 0; }
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* ----------------------------------------------------------------------------------- */
/* Set-up: AO CSR, groups, neighbour maps (section 3.2), Jacobi schedule (section 3.5) */

static int build_ao_csr(orc_t* o) {
  const int na = o->n_atoms;
  o->rp = xcalloc(o->n_ao + 1, sizeof(int64_t));
  for (int a = 0; a < na; ++a) {
    int64_t w = 0;
    for (int64_t k = o->blk_rowptr[a]; k < o->blk_rowptr[a + 1]; ++k) w += o->atom_nao[o->blk_col[k]];
    for (int r = 0; r < o->atom_nao[a]; ++r) o->rp[o->ao_off[a] + r + 1] = w;
  }
  for (int mu = 0; mu < o->n_ao; ++mu) o->rp[mu + 1] += o->rp[mu];
  const int64_t nnz = o->rp[o->n_ao];
  o->ci = xcalloc(nnz, sizeof(int32_t));
  o->ao2blk = xcalloc(nnz, sizeof(int64_t));
  o->S = xcalloc(nnz, sizeof(double));
  o->H0 = xcalloc(nnz, sizeof(double));
  o->H = xcalloc(nnz, sizeof(double));
  if (!o->ci || !o->ao2blk || !o->S || !o->H0 || !o->H) return ORC_E_ALLOC;
  return ORC_OK;
}

static void fill_ao_csr(orc_t* o, const double* Sv, const double* Hv) {
  for (int a = 0; a < o->n_atoms; ++a) {
    const int nra = o->atom_nao[a];
    for (int r = 0; r < nra; ++r) {
      const int32_t mu = (int32_t)(o->ao_off[a] + r);
      int64_t p = o->rp[mu];
      for (int64_t k = o->blk_rowptr[a]; k < o->blk_rowptr[a + 1]; ++k) {
        const int b = o->blk_col[k];
        const int nb = o->atom_nao[b];
        for (int c = 0; c < nb; ++c) {
          const int64_t src = o->blk_off[k] + (int64_t)r * nb + c;
          o->ci[p] = (int32_t)(o->ao_off[b] + c);
          o->ao2blk[p] = src;
          if (Sv) o->S[p] = Sv[src];
          if (Hv) o->H0[p] = Hv[src];
          ++p;
        }
      }
    }
  }
}

static int check_symmetric(const orc_t* o, const double* X) {
  for (int mu = 0; mu < o->n_ao; ++mu) {
    for (int64_t k = o->rp[mu]; k < o->rp[mu + 1]; ++k) {
      const int nu = o->ci[k];
      /* find (nu, mu) */
      int64_t lo = o->rp[nu], hi = o->rp[nu + 1] - 1, hit = -1;
      while (lo <= hi) {
        int64_t m = (lo + hi) / 2;
        if (o->ci[m] == mu) { hit = m; break; }
        if (o->ci[m] < mu) lo = m + 1; else hi = m - 1;
      }
      if (hit < 0 || X[hit] != X[k]) return 0;
    }
  }
  return 1;
}

/* Groups g and h are neighbours when some atom of g and some atom of h are
 * closer than r_nbr (section 3.2).  g ~ g always. */
static void build_group_nbr(orc_t* o) {
  const int G = o->n_groups;
  o->gnbr = xcalloc((size_t)G * G, 1);
  int32_t* ga_ptr = xcalloc(G + 1, sizeof(int32_t));
  int32_t* ga = xcalloc(o->n_atoms, sizeof(int32_t));
  for (int a = 0; a < o->n_atoms; ++a) ga_ptr[o->atom_group[a] + 1]++;
  for (int g = 0; g < G; ++g) ga_ptr[g + 1] += ga_ptr[g];
  int32_t* fillp = xcalloc(G, sizeof(int32_t));
  for (int a = 0; a < o->n_atoms; ++a) { int g = o->atom_group[a]; ga[ga_ptr[g] + fillp[g]++] = a; }
  const double r2 = o->r_nbr * o->r_nbr;
#pragma omp parallel for schedule(dynamic)
  for (int g = 0; g < G; ++g) {
    o->gnbr[(size_t)g * G + g] = 1;
    for (int t = ga_ptr[g]; t < ga_ptr[g + 1]; ++t) {
      const int a = ga[t];
      for (int b = 0; b < o->n_atoms; ++b) {
        const double dx = o->xyz[3 * a] - o->xyz[3 * b];
        const double dy = o->xyz[3 * a + 1] - o->xyz[3 * b + 1];
        const double dz = o->xyz[3 * a + 2] - o->xyz[3 * b + 2];
        if (dx * dx + dy * dy + dz * dz < r2) o->gnbr[(size_t)g * G + o->atom_group[b]] = 1;
      }
    }
  }
  free(ga_ptr); free(ga); free(fillp);
  o->gn_ptr = xcalloc(G + 1, sizeof(int32_t));
  for (int g = 0; g < G; ++g)
    for (int h = 0; h < G; ++h) o->gn_ptr[g + 1] += o->gnbr[(size_t)g * G + h];
  for (int g = 0; g < G; ++g) o->gn_ptr[g + 1] += o->gn_ptr[g];
  o->gn = xcalloc(o->gn_ptr[G], sizeof(int32_t));
  o->gn_pos = xcalloc((size_t)G * G, sizeof(int32_t));
  for (int g = 0; g < G; ++g) {
    int k = 0;
    for (int h = 0; h < G; ++h) {
      o->gn_pos[(size_t)g * G + h] = -1;
      if (o->gnbr[(size_t)g * G + h]) { o->gn[o->gn_ptr[g] + k] = h; o->gn_pos[(size_t)g * G + h] = k; ++k; }
    }
  }
}

/* Occupied-virtual blocks (g occupied, h virtual) between neighbouring groups,
 * coloured into rounds so that no two blocks of a round share a group's
 * occupied or virtual MOs: visit blocks in (g, h) order and give each the
 * smallest round not yet used by its g or its h (section 3.5 and its figure). */
static void build_schedule(orc_t* o) {
  const int G = o->n_groups;
  o->n_blocks = 0;
  for (int g = 0; g < G; ++g) {
    if (o->g_nocc[g] == 0) continue;
    for (int k = o->gn_ptr[g]; k < o->gn_ptr[g + 1]; ++k) {
      const int h = o->gn[k];
      const int nv = (o->gm_ptr[h + 1] - o->gm_ptr[h]) - o->g_nocc[h];
      if (nv > 0) o->n_blocks++;
    }
  }
  const int nb = o->n_blocks;
  o->jb_g = xcalloc(nb, sizeof(int32_t));
  o->jb_h = xcalloc(nb, sizeof(int32_t));
  o->jb_round = xcalloc(nb, sizeof(int32_t));
  o->jb_of = xcalloc((size_t)G * G, sizeof(int32_t));
  o->jb_foff = xcalloc(nb + 1, sizeof(int64_t));
  for (size_t t = 0; t < (size_t)G * G; ++t) o->jb_of[t] = -1;
  int maxdeg = 0;
  for (int g = 0; g < G; ++g) if (o->gn_ptr[g + 1] - o->gn_ptr[g] > maxdeg) maxdeg = o->gn_ptr[g + 1] - o->gn_ptr[g];
  const int RMAX = 2 * maxdeg + 2;
  uint8_t* used_o = xcalloc((size_t)G * RMAX, 1);
  uint8_t* used_v = xcalloc((size_t)G * RMAX, 1);
  int b = 0;
  o->n_rounds = 0;
  for (int g = 0; g < G; ++g) {
    if (o->g_nocc[g] == 0) continue;
    for (int k = o->gn_ptr[g]; k < o->gn_ptr[g + 1]; ++k) {
      const int h = o->gn[k];
      const int nv = (o->gm_ptr[h + 1] - o->gm_ptr[h]) - o->g_nocc[h];
      if (nv <= 0) continue;
      int r = 0;
      while (used_o[(size_t)g * RMAX + r] || used_v[(size_t)h * RMAX + r]) ++r;
      used_o[(size_t)g * RMAX + r] = 1;
      used_v[(size_t)h * RMAX + r] = 1;
      o->jb_g[b] = g; o->jb_h[b] = h; o->jb_round[b] = r;
      o->jb_of[(size_t)g * G + h] = b;
      o->jb_foff[b + 1] = o->jb_foff[b] + (int64_t)o->g_nocc[g] * nv;
      if (r + 1 > o->n_rounds) o->n_rounds = r + 1;
      ++b;
    }
  }
  free(used_o); free(used_v);
  o->F = xcalloc(o->jb_foff[nb], sizeof(double));
}

/* ----------------------------------------------------------------------------------- */
/* C^T S C over neighbouring groups (section 3.4 step b, section 3.6)               */

static double* oblk(const orc_t* o, int g, int h) {
  const int k = o->gn_pos[(size_t)g * o->n_groups + h];
  return o->O + o->ob_off[o->gn_ptr[g] + k];
}

static int n_in_group(const orc_t* o, int g) { return o->gm_ptr[g + 1] - o->gm_ptr[g]; }

/* O_ij = C_i^T S C_j for i, j in neighbouring groups; O_ij is computed once (i <= j)
 * and stored in both blocks.  only_occ restricts to occupied pairs. */
static void overlap_mo(orc_t* o, int only_occ) {
  const int n_scope = only_occ ? o->n_occ : o->n_mo;
#pragma omp parallel
  {
    double* y = xcalloc(o->n_ao, sizeof(double));
    uint8_t* mark = xcalloc(o->n_ao, 1);
    int32_t* list = xcalloc(o->n_ao, sizeof(int32_t));
#pragma omp for schedule(dynamic, 4)
    for (int j = 0; j < n_scope; ++j) {
      const int32_t nt = spmv_col(o, o->S, &o->C[j], y, mark, list);
      const int h = o->mo_group[j];
      const int jl = o->mo_local[j];
      const int nh = n_in_group(o, h);
      for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) {
        const int g = o->gn[k];
        const int ng = n_in_group(o, g);
        double* Ogh = oblk(o, g, h);
        double* Ohg = oblk(o, h, g);
        for (int il = 0; il < ng; ++il) {
          const int i = o->gm[o->gm_ptr[g] + il];
          if (i > j) break;          /* MOs of a group are ascending */
          if (i >= n_scope) break;
          const double v = col_dot_dense(&o->C[i], y);
          Ogh[(size_t)il * nh + jl] = v;
          Ohg[(size_t)jl * ng + il] = v;
        }
      }
      clear_touched(y, mark, list, nt);
    }
    free(y); free(mark); free(list);
  }
}

/* ----------------------------------------------------------------------------------- */
/* Work accounting (measurement only; see orc_work in oracle.h).  Each function counts  */
/* one pass on the current state and adds to o->work; none changes a value.            */

static int64_t count_nonzero(const double* x, int64_t n) {
  int64_t c = 0;
  for (int64_t t = 0; t < n; ++t) c += x[t] != 0.0;
  return c;
}

static int64_t col_nnz(const col_t* c) { return count_nonzero(c->val, c->n); }

/* nonzeros of row nu of the AO matrix X */
static int64_t x_row_nnz(const orc_t* o, const double* X, int nu) {
  return count_nonzero(X + o->rp[nu], o->rp[nu + 1] - o->rp[nu]);
}

/* Y = X C over MOs [0, n_scope) */
static void work_product(orc_t* o, const double* X, int n_scope) {
  const int64_t nnz_x = count_nonzero(X, o->rp[o->n_ao]);
  double fl = 0.0, nc = 0.0, ny = 0.0;
#pragma omp parallel reduction(+ : fl, nc, ny)
  {
    double* y = xcalloc(o->n_ao, sizeof(double));
    uint8_t* mark = xcalloc(o->n_ao, 1);
    int32_t* list = xcalloc(o->n_ao, sizeof(int32_t));
#pragma omp for schedule(dynamic, 16)
    for (int j = 0; j < n_scope; ++j) {
      const col_t* c = &o->C[j];
      for (int32_t t = 0; t < c->n; ++t)
        if (c->val[t] != 0.0) { fl += (double)x_row_nnz(o, X, c->row[t]); nc += 1.0; }
      const int32_t nt = spmv_col(o, X, c, y, mark, list);
      for (int32_t t = 0; t < nt; ++t) ny += y[list[t]] != 0.0;
      clear_touched(y, mark, list, nt);
    }
    free(y); free(mark); free(list);
  }
  o->work.flops[ORC_W_PRODUCT] += 2.0 * fl;
  o->work.bytes[ORC_W_PRODUCT] += 8.0 * ((double)nnz_x + nc + ny);
  o->work.passes[ORC_W_PRODUCT] += 1;
}

/* |supp C_i ∩ supp y| for a dense y */
static int64_t support_meet(const col_t* c, const double* y) {
  int64_t k = 0;
  for (int32_t t = 0; t < c->n; ++t) k += c->val[t] != 0.0 && y[c->row[t]] != 0.0;
  return k;
}

/* C^T S C pairs (only_occ: occupied MOs): for neighbouring groups g <= h, i in g and j in h,
 * with local(i) <= local(j) when g == h */
static void work_overlap(orc_t* o, int n_scope) {
  double fl = 0.0, nc = 0.0, ny = 0.0, np = 0.0;
#pragma omp parallel reduction(+ : fl, nc, ny, np)
  {
    double* y = xcalloc(o->n_ao, sizeof(double));
    uint8_t* mark = xcalloc(o->n_ao, 1);
    int32_t* list = xcalloc(o->n_ao, sizeof(int32_t));
#pragma omp for schedule(dynamic, 4)
    for (int j = 0; j < n_scope; ++j) {
      nc += (double)col_nnz(&o->C[j]);
      const int32_t nt = spmv_col(o, o->S, &o->C[j], y, mark, list);
      for (int32_t t = 0; t < nt; ++t) ny += y[list[t]] != 0.0;
      const int h = o->mo_group[j], jl = o->mo_local[j];
      for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) {
        const int g = o->gn[k];
        if (g > h) continue;
        for (int il = 0; il < n_in_group(o, g); ++il) {
          const int i = o->gm[o->gm_ptr[g] + il];
          if (i >= n_scope || (g == h && il > jl)) continue;
          fl += (double)support_meet(&o->C[i], y);
          np += 1.0;
        }
      }
      clear_touched(y, mark, list, nt);
    }
    free(y); free(mark); free(list);
  }
  o->work.flops[ORC_W_OVERLAP] += 2.0 * fl;
  o->work.bytes[ORC_W_OVERLAP] += 8.0 * (nc + ny + np);
  o->work.passes[ORC_W_OVERLAP] += 1;
}

/* occupied-virtual C_i^T (H C)_a of the Jacobi blocks */
static void work_fock_blocks(orc_t* o) {
  const int G = o->n_groups;
  double fl = 0.0, nc = 0.0, ny = 0.0, np = 0.0;
  for (int i = 0; i < o->n_occ; ++i) nc += (double)col_nnz(&o->C[i]);
#pragma omp parallel reduction(+ : fl, ny, np)
  {
    double* y = xcalloc(o->n_ao, sizeof(double));
    uint8_t* mark = xcalloc(o->n_ao, 1);
    int32_t* list = xcalloc(o->n_ao, sizeof(int32_t));
#pragma omp for schedule(dynamic, 4)
    for (int a = o->n_occ; a < o->n_mo; ++a) {
      const int32_t nt = spmv_col(o, o->H, &o->C[a], y, mark, list);
      for (int32_t t = 0; t < nt; ++t) ny += y[list[t]] != 0.0;
      const int h = o->mo_group[a];
      for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) {
        const int g = o->gn[k];
        if (o->jb_of[(size_t)g * G + h] < 0) continue;
        for (int il = 0; il < o->g_nocc[g]; ++il) {
          fl += (double)support_meet(&o->C[o->gm[o->gm_ptr[g] + il]], y);
          np += 1.0;
        }
      }
      clear_touched(y, mark, list, nt);
    }
    free(y); free(mark); free(list);
  }
  o->work.flops[ORC_W_FOCK_BLOCKS] += 2.0 * fl;
  o->work.bytes[ORC_W_FOCK_BLOCKS] += 8.0 * (nc + ny + np);
  o->work.passes[ORC_W_FOCK_BLOCKS] += 1;
}

static int64_t nnz_scope(const orc_t* o, int n_scope) {
  int64_t n = 0;
  for (int j = 0; j < n_scope; ++j) n += col_nnz(&o->C[j]);
  return n;
}

/* the selected pairs of a combination sweep, before it runs (D in o->O, threshold thr);
 * with the trace on, C entering and the pair list are kept */
static void work_combine_begin(orc_t* o, int n_scope, double thr, double eta) {
  double fl = 0.0, ns = 0.0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : fl, ns)
  for (int j = 0; j < n_scope; ++j) {
    const int h = o->mo_group[j], jl = o->mo_local[j], nh = n_in_group(o, h);
    for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) {
      const int g = o->gn[k];
      const double* Dgh = oblk(o, g, h);
      for (int il = 0; il < n_in_group(o, g); ++il) {
        const int i = o->gm[o->gm_ptr[g] + il];
        if (i >= n_scope || i == j) continue;
        if (fabs(Dgh[(size_t)il * nh + jl]) < thr) continue;
        ns += 1.0;
        fl += (double)col_nnz(&o->C[i]);
      }
    }
  }
  const int64_t nin = nnz_scope(o, n_scope);
  o->work.flops[ORC_W_COMBINE] += 2.0 * fl;
  o->work.bytes[ORC_W_COMBINE] += 8.0 * ((double)nin + ns);
  o->work.passes[ORC_W_COMBINE] += 1;
  const int k = o->work.n_sweeps;
  if (k < ORC_W_MAX_SWEEPS) {
    o->work.sweep_sel[k] = (int64_t)ns;
    o->work.sweep_nnz_in[k] = nin;
    o->work.sweep_flops[k] = 2.0 * fl;
  }
  if (o->trace_on) {
    if (o->n_trace == o->cap_trace) {
      o->cap_trace = o->cap_trace ? 2 * o->cap_trace : 8;
      o->trace = realloc(o->trace, sizeof(struct trace_sweep) * o->cap_trace);
    }
    struct trace_sweep* t = &o->trace[o->n_trace++];
    memset(t, 0, sizeof(*t));
    t->n_scope = n_scope;
    t->eta = eta;
    t->colptr = xcalloc(n_scope + 1, sizeof(int64_t));
    for (int j = 0; j < n_scope; ++j) t->colptr[j + 1] = t->colptr[j] + o->C[j].n;
    t->nnz = t->colptr[n_scope];
    t->row = xcalloc(t->nnz, sizeof(int32_t));
    t->val = xcalloc(t->nnz, sizeof(double));
    for (int j = 0; j < n_scope; ++j) {
      memcpy(t->row + t->colptr[j], o->C[j].row, sizeof(int32_t) * o->C[j].n);
      memcpy(t->val + t->colptr[j], o->C[j].val, sizeof(double) * o->C[j].n);
    }
    t->n_sel = (int64_t)ns;
    t->si = xcalloc(t->n_sel, sizeof(int32_t));
    t->sj = xcalloc(t->n_sel, sizeof(int32_t));
    t->sd = xcalloc(t->n_sel, sizeof(double));
    int64_t w = 0;
    for (int j = 0; j < n_scope; ++j) {
      const int h = o->mo_group[j], jl = o->mo_local[j], nh = n_in_group(o, h);
      for (int k2 = o->gn_ptr[h]; k2 < o->gn_ptr[h + 1]; ++k2) {
        const int g = o->gn[k2];
        const double* Dgh = oblk(o, g, h);
        for (int il = 0; il < n_in_group(o, g); ++il) {
          const int i = o->gm[o->gm_ptr[g] + il];
          const double d = Dgh[(size_t)il * nh + jl];
          if (i >= n_scope || i == j || fabs(d) < thr) continue;
          t->si[w] = i; t->sj[w] = j; t->sd[w] = d; ++w;
        }
      }
    }
  }
}

static void work_combine_end(orc_t* o, int n_scope) {
  const int64_t nout = nnz_scope(o, n_scope);
  o->work.bytes[ORC_W_COMBINE] += 8.0 * (double)nout;
  if (o->work.n_sweeps < ORC_W_MAX_SWEEPS) o->work.sweep_nnz_out[o->work.n_sweeps] = nout;
  o->work.n_sweeps += 1;
}

static void trace_clear(orc_t* o) {
  for (int k = 0; k < o->n_trace; ++k) {
    struct trace_sweep* t = &o->trace[k];
    free(t->colptr); free(t->row); free(t->val); free(t->si); free(t->sj); free(t->sd);
  }
  o->n_trace = 0;
}

static void work_reset(orc_t* o) {
  memset(&o->work, 0, sizeof(o->work));
  trace_clear(o);
}

/* Orthonormalization loop (section 3.4; thresholds of section 4.1).
 * Returns ORC_OK, ORC_E_NOT_SPD; *converged tells whether eta < eps/100 was reached. */
/* The section's combination taken literally: every selected pair (i, j), i < j, in
 * ascending order, combined from the two columns as they stand at that moment,
 * C'_i = C_i - 1/2 D_ij C_j and C'_j = C_j - 1/2 D_ij C_i, and the pair's two columns cut at
 * |C| < cut right away.  Sequential; for quantifying the simultaneous reading only. */
static void combine_pairs_in_order(orc_t* o, int n_scope, double thr, double cut) {
  double* yi = xcalloc(o->n_ao, sizeof(double));
  double* yj = xcalloc(o->n_ao, sizeof(double));
  uint8_t* mark = xcalloc(o->n_ao, 1);
  int32_t* list = xcalloc(o->n_ao, sizeof(int32_t));
  for (int i = 0; i < n_scope; ++i) {
    const int g = o->mo_group[i], il = o->mo_local[i], ng = n_in_group(o, g);
    (void)ng;
    for (int j = i + 1; j < n_scope; ++j) {
      const int h = o->mo_group[j], jl = o->mo_local[j], nh = n_in_group(o, h);
      int nbr = 0;
      for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) if (o->gn[k] == g) { nbr = 1; break; }
      if (!nbr) continue;
      const double d = oblk(o, g, h)[(size_t)il * nh + jl];
      if (fabs(d) < thr) continue;
      int32_t nt = 0;
      for (int32_t t = 0; t < o->C[i].n; ++t) {
        const int32_t mu = o->C[i].row[t];
        if (!mark[mu]) { mark[mu] = 1; list[nt++] = mu; }
        yi[mu] = o->C[i].val[t];
      }
      for (int32_t t = 0; t < o->C[j].n; ++t) {
        const int32_t mu = o->C[j].row[t];
        if (!mark[mu]) { mark[mu] = 1; list[nt++] = mu; }
        yj[mu] = o->C[j].val[t];
      }
      qsort(list, nt, sizeof(int32_t), cmp_i32);
      int32_t ki = 0, kj = 0;
      for (int32_t t = 0; t < nt; ++t) {
        const int32_t mu = list[t];
        const double xi = yi[mu], xj = yj[mu];
        yi[mu] = xi - 0.5 * d * xj;
        yj[mu] = xj - 0.5 * d * xi;
        ki += fabs(yi[mu]) >= cut;
        kj += fabs(yj[mu]) >= cut;
      }
      col_t* ci = &o->C[i];
      col_t* cj = &o->C[j];
      col_free(ci);
      col_free(cj);
      ci->n = ki; ci->row = malloc(sizeof(int32_t) * (ki ? ki : 1)); ci->val = malloc(sizeof(double) * (ki ? ki : 1));
      cj->n = kj; cj->row = malloc(sizeof(int32_t) * (kj ? kj : 1)); cj->val = malloc(sizeof(double) * (kj ? kj : 1));
      int32_t wi = 0, wj = 0;
      for (int32_t t = 0; t < nt; ++t) {
        const int32_t mu = list[t];
        if (fabs(yi[mu]) >= cut) { ci->row[wi] = mu; ci->val[wi] = yi[mu]; ++wi; }
        if (fabs(yj[mu]) >= cut) { cj->row[wj] = mu; cj->val[wj] = yj[mu]; ++wj; }
        yi[mu] = 0.0; yj[mu] = 0.0; mark[mu] = 0;
      }
    }
  }
  free(yi); free(yj); free(mark); free(list);
}

static int orthonormalize(orc_t* o, int only_occ, int max_sweeps, int* sweeps_out,
                          double* eta_out, int* converged) {
  const int n_scope = only_occ ? o->n_occ : o->n_mo;
  const double tol = o->eps / 100.0;
  const double cut = 1e-3 * o->eps;
  double* sc = xcalloc(n_scope, sizeof(double));
  col_t* Cn = xcalloc(n_scope, sizeof(col_t));
  int sweeps = 0;
  double eta = 0.0;
  *converged = 0;
  for (;;) {
    if (o->count_on) {
      work_product(o, o->S, n_scope);
      work_overlap(o, n_scope);
    }
    overlap_mo(o, only_occ);
    /* normalize with the diagonal */
    int bad = 0;
    for (int j = 0; j < n_scope; ++j) {
      const int g = o->mo_group[j], jl = o->mo_local[j], ng = n_in_group(o, g);
      const double d = oblk(o, g, g)[(size_t)jl * ng + jl];
      if (!(d > 0.0)) bad = 1;
      sc[j] = sqrt(d);
    }
    if (bad) { free(sc); free(Cn); return fail(o, ORC_E_NOT_SPD, "C^T S C has a non-positive diagonal"); }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n_scope; ++j)
      for (int32_t t = 0; t < o->C[j].n; ++t) o->C[j].val[t] /= sc[j];
    /* D_ij = O_ij / sqrt(O_ii O_jj) in place, eta = max |D_ij| over i != j */
    eta = 0.0;
#pragma omp parallel for schedule(dynamic) reduction(max : eta)
    for (int j = 0; j < n_scope; ++j) {
      const int h = o->mo_group[j], jl = o->mo_local[j], nh = n_in_group(o, h);
      for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) {
        const int g = o->gn[k], ng = n_in_group(o, g);
        double* Ogh = oblk(o, g, h);
        for (int il = 0; il < ng; ++il) {
          const int i = o->gm[o->gm_ptr[g] + il];
          if (i >= n_scope) break;
          double* e = &Ogh[(size_t)il * nh + jl];
          if (i == j) { *e = 1.0; continue; }
          *e = *e / (sc[i] * sc[j]);
          if (fabs(*e) > eta) eta = fabs(*e);
        }
      }
    }
    if (eta < tol) { *converged = 1; break; }
    if (sweeps >= max_sweeps) break;
    /* pair combinations C'_j = C_j - 1/2 sum_i C_i D_ij over |D_ij| >= 1e-3 eta */
    const double thr = 1e-3 * eta;
    if (o->literal_ortho) {
      combine_pairs_in_order(o, n_scope, thr, cut);
      ++sweeps;
      continue;
    }
    if (o->count_on || o->trace_on) work_combine_begin(o, n_scope, thr, eta);
#pragma omp parallel
    {
      double* y = xcalloc(o->n_ao, sizeof(double));
      uint8_t* mark = xcalloc(o->n_ao, 1);
      int32_t* list = xcalloc(o->n_ao, sizeof(int32_t));
#pragma omp for schedule(dynamic, 4)
      for (int j = 0; j < n_scope; ++j) {
        const int h = o->mo_group[j], jl = o->mo_local[j], nh = n_in_group(o, h);
        int32_t nt = 0;
        for (int32_t t = 0; t < o->C[j].n; ++t) {
          const int32_t mu = o->C[j].row[t];
          mark[mu] = 1; list[nt++] = mu; y[mu] = o->C[j].val[t];
        }
        int updated = 0;
        for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) {
          const int g = o->gn[k], ng = n_in_group(o, g);
          const double* Dgh = oblk(o, g, h);
          for (int il = 0; il < ng; ++il) {
            const int i = o->gm[o->gm_ptr[g] + il];
            if (i >= n_scope) break;
            if (i == j) continue;
            const double d = Dgh[(size_t)il * nh + jl];
            if (fabs(d) < thr) continue;
            updated = 1;
            const double f = -0.5 * d;
            for (int32_t t = 0; t < o->C[i].n; ++t) {
              const int32_t mu = o->C[i].row[t];
              if (!mark[mu]) { mark[mu] = 1; list[nt++] = mu; y[mu] = 0.0; }
              y[mu] += f * o->C[i].val[t];
            }
          }
        }
        qsort(list, nt, sizeof(int32_t), cmp_i32);
        int32_t keep = 0;
        for (int32_t t = 0; t < nt; ++t)
          if (!updated || fabs(y[list[t]]) >= cut) ++keep;
        Cn[j].n = keep;
        Cn[j].row = malloc(sizeof(int32_t) * (keep ? keep : 1));
        Cn[j].val = malloc(sizeof(double) * (keep ? keep : 1));
        int32_t w = 0;
        for (int32_t t = 0; t < nt; ++t) {
          const int32_t mu = list[t];
          const double v = y[mu];
          if (!updated || fabs(v) >= cut) { Cn[j].row[w] = mu; Cn[j].val[w] = v; ++w; }
          y[mu] = 0.0; mark[mu] = 0;
        }
      }
      free(y); free(mark); free(list);
    }
    for (int j = 0; j < n_scope; ++j) { col_free(&o->C[j]); o->C[j] = Cn[j]; Cn[j].row = NULL; Cn[j].val = NULL; Cn[j].n = 0; }
    if (o->count_on || o->trace_on) work_combine_end(o, n_scope);
    ++sweeps;
  }
  free(sc); free(Cn);
  *sweeps_out = sweeps;
  *eta_out = eta;
  return ORC_OK;
}

/* ----------------------------------------------------------------------------------- */
/* DFTB Fock matrix (section 3.7)                                                    */

static double gamma_ab(const orc_t* o, int a, int b) {
  if (a == b) return o->U[a];
  const double dx = o->xyz[3 * a] - o->xyz[3 * b];
  const double dy = o->xyz[3 * a + 1] - o->xyz[3 * b + 1];
  const double dz = o->xyz[3 * a + 2] - o->xyz[3 * b + 2];
  const double u = 0.5 * (1.0 / o->U[a] + 1.0 / o->U[b]);
  return 1.0 / sqrt(dx * dx + dy * dy + dz * dz + u * u);
}

/* Q_a = sum_x gamma_ax dq_x over every atom pair, unscreened */
static void coulomb_q(orc_t* o) {
#pragma omp parallel for schedule(static)
  for (int a = 0; a < o->n_atoms; ++a) {
    double s = 0.0;
    if (o->scc)
      for (int x = 0; x < o->n_atoms; ++x) s += gamma_ab(o, a, x) * o->dq[x];
    o->Q[a] = s;
  }
}

/* H_uv = H0_uv + 1/2 S_uv (Q_a + Q_b), then |H_uv| < eps -> 0 (section 4.1) */
static void fock_build(orc_t* o) {
#pragma omp parallel for schedule(static)
  for (int mu = 0; mu < o->n_ao; ++mu) {
    const double qa = o->Q[o->ao_atom[mu]];
    for (int64_t k = o->rp[mu]; k < o->rp[mu + 1]; ++k) {
      double h;
      if (o->fock_full) h = o->Fuser[k];
      else h = o->H0[k] + 0.5 * o->S[k] * (qa + o->Q[o->ao_atom[o->ci[k]]]);
      o->H[k] = (fabs(h) < o->eps) ? 0.0 : h;
    }
  }
}

/* ----------------------------------------------------------------------------------- */
/* C^T H C: occupied-virtual blocks of neighbouring groups and the diagonal          */

static double fmo(orc_t* o) {
  const int G = o->n_groups;
#pragma omp parallel
  {
    double* y = xcalloc(o->n_ao, sizeof(double));
    uint8_t* mark = xcalloc(o->n_ao, 1);
    int32_t* list = xcalloc(o->n_ao, sizeof(int32_t));
#pragma omp for schedule(dynamic, 4)
    for (int j = 0; j < o->n_mo; ++j) {
      const int32_t nt = spmv_col(o, o->H, &o->C[j], y, mark, list);
      o->Fdiag[j] = col_dot_dense(&o->C[j], y);
      if (j >= o->n_occ) {
        const int h = o->mo_group[j];
        const int al = o->mo_local[j] - o->g_nocc[h];
        const int nv = n_in_group(o, h) - o->g_nocc[h];
        for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) {
          const int g = o->gn[k];
          const int b = o->jb_of[(size_t)g * G + h];
          if (b < 0) continue;
          double* Fb = o->F + o->jb_foff[b];
          for (int il = 0; il < o->g_nocc[g]; ++il) {
            const int i = o->gm[o->gm_ptr[g] + il];
            Fb[(size_t)il * nv + al] = col_dot_dense(&o->C[i], y);
          }
        }
      }
      clear_touched(y, mark, list, nt);
    }
    free(y); free(mark); free(list);
  }
  double m = 0.0;
  for (int64_t t = 0; t < o->jb_foff[o->n_blocks]; ++t) if (fabs(o->F[t]) > m) m = fabs(o->F[t]);
  return m;
}

/* ----------------------------------------------------------------------------------- */
/* Rotation selection (section 3.5 steps 3-4)                                        */

void orc_jacobi_angle(double fii, double faa, double fia, double* c, double* s) {
  const double p = (fii - faa) / (2.0 * fia);
  const double sg = (p >= 0.0) ? 1.0 : -1.0;
  const double t = 1.0 / (p + sg * sqrt(1.0 + p * p));
  *c = 1.0 / sqrt(1.0 + t * t);
  *s = t * (*c);
}

typedef struct {
  double af;
  int32_t i, a, b, round;
  double f;
} cand_t;

static int cmp_cand_size(const void* x, const void* y) {
  const cand_t* p = x; const cand_t* q = y;
  if (p->af != q->af) return (p->af > q->af) ? -1 : 1;
  if (p->i != q->i) return (p->i < q->i) ? -1 : 1;
  return (p->a < q->a) ? -1 : (p->a > q->a);
}

static int cmp_cand_order(const void* x, const void* y) {
  const cand_t* p = x; const cand_t* q = y;
  if (p->round != q->round) return (p->round < q->round) ? -1 : 1;
  if (p->b != q->b) return (p->b < q->b) ? -1 : 1;
  return cmp_cand_size(x, y);
}

static int select_rotations(orc_t* o) {
  int64_t n = 0;
  for (int b = 0; b < o->n_blocks; ++b) {
    const double* Fb = o->F + o->jb_foff[b];
    for (int64_t t = 0; t < o->jb_foff[b + 1] - o->jb_foff[b]; ++t)
      if (Fb[t] != 0.0 && fabs(Fb[t]) >= o->eps) ++n;
  }
  cand_t* cd = xcalloc(n, sizeof(cand_t));
  int64_t w = 0;
  for (int b = 0; b < o->n_blocks; ++b) {
    const int g = o->jb_g[b], h = o->jb_h[b];
    const int nv = n_in_group(o, h) - o->g_nocc[h];
    const double* Fb = o->F + o->jb_foff[b];
    for (int il = 0; il < o->g_nocc[g]; ++il)
      for (int al = 0; al < nv; ++al) {
        const double f = Fb[(size_t)il * nv + al];
        if (f == 0.0 || fabs(f) < o->eps) continue;
        cd[w].af = fabs(f); cd[w].f = f; cd[w].b = b; cd[w].round = o->jb_round[b];
        cd[w].i = o->gm[o->gm_ptr[g] + il];
        cd[w].a = o->gm[o->gm_ptr[h] + o->g_nocc[h] + al];
        ++w;
      }
  }
  const int64_t K = (int64_t)floor(o->rot_cap_factor * o->n_occ);
  int64_t nk = n;
  if (n > K) { qsort(cd, n, sizeof(cand_t), cmp_cand_size); nk = K; }
  qsort(cd, nk, sizeof(cand_t), cmp_cand_order);
  free(o->rot_i); free(o->rot_a); free(o->rot_c); free(o->rot_s); free(o->rot_blk);
  o->rot_i = xcalloc(nk, sizeof(int32_t)); o->rot_a = xcalloc(nk, sizeof(int32_t));
  o->rot_c = xcalloc(nk, sizeof(double)); o->rot_s = xcalloc(nk, sizeof(double));
  o->rot_blk = xcalloc(nk, sizeof(int32_t));
  for (int64_t t = 0; t < nk; ++t) {
    o->rot_i[t] = cd[t].i; o->rot_a[t] = cd[t].a; o->rot_blk[t] = cd[t].b;
    orc_jacobi_angle(o->Fdiag[cd[t].i], o->Fdiag[cd[t].a], cd[t].f, &o->rot_c[t], &o->rot_s[t]);
  }
  o->n_rot = (int)nk;
  free(cd);
  return (int)n;
}

/* Apply the ordered rotations: C'_i = c C_i + s C_a, C'_a = -s C_i + c C_a; after
 * each block, zero |C_ki| < eps in the columns it rotated.  Blocks of one round
 * share no MO and are independent. */
static void apply_rotations(orc_t* o) {
  /* each block's rotations form one contiguous run [rb0[b], rb1[b]) of the list,
   * which is ordered by round, then block */
  int32_t* rb0 = xcalloc(o->n_blocks, sizeof(int32_t));
  int32_t* rb1 = xcalloc(o->n_blocks, sizeof(int32_t));
  for (int t = 0; t < o->n_rot; ++t) {
    const int b = o->rot_blk[t];
    if (t == 0 || o->rot_blk[t - 1] != b) rb0[b] = t;
    rb1[b] = t + 1;
  }
  int32_t* blist = xcalloc(o->n_blocks, sizeof(int32_t));
  double w_flops = 0.0, w_bytes = 0.0;      /* work accounting (orc_set_count) */
  for (int r = 0; r < o->n_rounds; ++r) {
    int nbl = 0;
    for (int b = 0; b < o->n_blocks; ++b)
      if (o->jb_round[b] == r && rb1[b] > rb0[b]) blist[nbl++] = b;
#pragma omp parallel
    {
      int32_t* pos = xcalloc(o->n_ao, sizeof(int32_t));
      int32_t* U = xcalloc(o->n_ao, sizeof(int32_t));
      int32_t* cols = xcalloc(2 * (size_t)o->n_rot + 2, sizeof(int32_t));
      for (int mu = 0; mu < o->n_ao; ++mu) pos[mu] = -1;
#pragma omp for schedule(dynamic)
      for (int bb = 0; bb < nbl; ++bb) {
        const int b = blist[bb];
        /* involved columns, ascending and unique */
        int nc = 0;
        for (int t = rb0[b]; t < rb1[b]; ++t) { cols[nc++] = o->rot_i[t]; cols[nc++] = o->rot_a[t]; }
        qsort(cols, nc, sizeof(int32_t), cmp_i32);
        int u = 0;
        for (int t = 0; t < nc; ++t) if (t == 0 || cols[t] != cols[t - 1]) cols[u++] = cols[t];
        nc = u;
        /* union of their rows */
        int32_t nu = 0;
        for (int t = 0; t < nc; ++t) {
          const col_t* c = &o->C[cols[t]];
          for (int32_t k = 0; k < c->n; ++k)
            if (pos[c->row[k]] < 0) { pos[c->row[k]] = 0; U[nu++] = c->row[k]; }
        }
        qsort(U, nu, sizeof(int32_t), cmp_i32);
        for (int32_t k = 0; k < nu; ++k) pos[U[k]] = k;
        if (o->count_on) {
          int64_t nz = 0;
          for (int t = 0; t < nc; ++t) nz += col_nnz(&o->C[cols[t]]);
#pragma omp atomic
          w_bytes += 16.0 * (double)nz;
#pragma omp atomic
          w_flops += 6.0 * (double)(rb1[b] - rb0[b]) * (double)nu;
        }
        double* v = xcalloc((size_t)nc * (nu ? nu : 1), sizeof(double));
        for (int t = 0; t < nc; ++t) {
          const col_t* c = &o->C[cols[t]];
          for (int32_t k = 0; k < c->n; ++k) v[(size_t)t * nu + pos[c->row[k]]] = c->val[k];
        }
        for (int t = rb0[b]; t < rb1[b]; ++t) {
          const int32_t* pi = bsearch(&o->rot_i[t], cols, nc, sizeof(int32_t), cmp_i32);
          const int32_t* pa = bsearch(&o->rot_a[t], cols, nc, sizeof(int32_t), cmp_i32);
          double* vi = v + (size_t)(pi - cols) * nu;
          double* va = v + (size_t)(pa - cols) * nu;
          const double c = o->rot_c[t], s = o->rot_s[t];
          for (int32_t k = 0; k < nu; ++k) {
            const double xi = vi[k], xa = va[k];
            vi[k] = c * xi + s * xa;
            va[k] = -s * xi + c * xa;
          }
          if (o->literal_rot)        /* truncation after every single rotation */
            for (int32_t k = 0; k < nu; ++k) {
              if (fabs(vi[k]) < o->eps) vi[k] = 0.0;
              if (fabs(va[k]) < o->eps) va[k] = 0.0;
            }
        }
        for (int t = 0; t < nc; ++t) {
          col_t* c = &o->C[cols[t]];
          const double* vt = v + (size_t)t * nu;
          int32_t keep = 0;
          for (int32_t k = 0; k < nu; ++k) if (fabs(vt[k]) >= o->eps) ++keep;
          col_free(c);
          c->n = keep;
          c->row = malloc(sizeof(int32_t) * (keep ? keep : 1));
          c->val = malloc(sizeof(double) * (keep ? keep : 1));
          int32_t w = 0;
          for (int32_t k = 0; k < nu; ++k)
            if (fabs(vt[k]) >= o->eps) { c->row[w] = U[k]; c->val[w] = vt[k]; ++w; }
        }
        for (int32_t k = 0; k < nu; ++k) pos[U[k]] = -1;
        free(v);
      }
      free(pos); free(U); free(cols);
    }
  }
  free(rb0); free(rb1); free(blist);
  if (o->count_on) {
    o->work.flops[ORC_W_ROTATE] += w_flops;
    o->work.bytes[ORC_W_ROTATE] += w_bytes;
    o->work.passes[ORC_W_ROTATE] += 1;
  }
}

/* ----------------------------------------------------------------------------------- */
/* Density, Mulliken charges (section 3.7, eq. pop) and energy                       */

static void density_charges(orc_t* o) {
  /* rows of C_occ: (i, C_ui) with i ascending */
  int64_t* rptr = xcalloc(o->n_ao + 1, sizeof(int64_t));
  for (int i = 0; i < o->n_occ; ++i)
    for (int32_t t = 0; t < o->C[i].n; ++t) rptr[o->C[i].row[t] + 1]++;
  for (int mu = 0; mu < o->n_ao; ++mu) rptr[mu + 1] += rptr[mu];
  int32_t* rmo = xcalloc(rptr[o->n_ao], sizeof(int32_t));
  double* rval = xcalloc(rptr[o->n_ao], sizeof(double));
  int64_t* fillp = xcalloc(o->n_ao, sizeof(int64_t));
  for (int i = 0; i < o->n_occ; ++i)
    for (int32_t t = 0; t < o->C[i].n; ++t) {
      const int mu = o->C[i].row[t];
      const int64_t p = rptr[mu] + fillp[mu]++;
      rmo[p] = i; rval[p] = o->C[i].val[t];
    }
  free(fillp);
  /* P_uv = 2 sum_i C_ui C_vi on the pattern of S */
#pragma omp parallel
  {
    double* w = xcalloc(o->n_occ, sizeof(double));
#pragma omp for schedule(dynamic, 16)
    for (int mu = 0; mu < o->n_ao; ++mu) {
      for (int64_t t = rptr[mu]; t < rptr[mu + 1]; ++t) w[rmo[t]] = rval[t];
      for (int64_t k = o->rp[mu]; k < o->rp[mu + 1]; ++k) {
        const int nu = o->ci[k];
        double s = 0.0;
        for (int64_t t = rptr[nu]; t < rptr[nu + 1]; ++t) s += w[rmo[t]] * rval[t];
        o->P[k] = 2.0 * s;
      }
      for (int64_t t = rptr[mu]; t < rptr[mu + 1]; ++t) w[rmo[t]] = 0.0;
    }
    free(w);
  }
  free(rptr); free(rmo); free(rval);
  /* q_a = sum_{u in a} sum_v P_uv S_uv */
#pragma omp parallel for schedule(static)
  for (int a = 0; a < o->n_atoms; ++a) {
    double s = 0.0;
    for (int64_t mu = o->ao_off[a]; mu < o->ao_off[a + 1]; ++mu)
      for (int64_t k = o->rp[mu]; k < o->rp[mu + 1]; ++k) s += o->P[k] * o->S[k];
    o->q[a] = s;
  }
  for (int a = 0; a < o->n_atoms; ++a) o->dq[a] = o->q[a] - o->q0[a];
}

static void energy(orc_t* o) {
  if (o->count_on) work_product(o, o->fock_full ? o->Fuser : o->H0, o->n_occ);
  coulomb_q(o);
  double* rs = xcalloc(o->n_ao, sizeof(double));
  const double* X = o->fock_full ? o->Fuser : o->H0;
#pragma omp parallel for schedule(static)
  for (int mu = 0; mu < o->n_ao; ++mu) {
    ksum_t k = {0, 0};
    for (int64_t t = o->rp[mu]; t < o->rp[mu + 1]; ++t) ks_add(&k, o->P[t] * X[t]);
    rs[mu] = ks_get(&k);
  }
  ksum_t kb = {0, 0}, kc = {0, 0};
  for (int mu = 0; mu < o->n_ao; ++mu) ks_add(&kb, rs[mu]);
  for (int a = 0; a < o->n_atoms; ++a) ks_add(&kc, 0.5 * o->dq[a] * o->Q[a]);
  free(rs);
  o->e_band = ks_get(&kb);
  o->e_coul = o->fock_full ? 0.0 : ks_get(&kc);
  o->E = o->e_band + o->e_coul;
}

/* ----------------------------------------------------------------------------------- */
/* Energy gradient at the current MOs (differentiation form).                          */
/* At self-consistency the energy of section 3.7 is stationary in the occupied MOs     */
/* under C^T S C = 1, and dE/dP = H (the Fock matrix of the current charges).  Hence   */
/*   dE/dX_uv = P_uv              (X = H0; with a complete Fock matrix, X = F)          */
/*   dE/dS_uv = -W_uv + 1/2 P_uv (Q_a + Q_b)   (the second term with the charge term)  */
/* where the first term of dE/dS comes from the orthonormality constraint and the      */
/* second from the S in the Mulliken charges (eq. pop).  W = 2 C_occ F C_occ^T with    */
/* F_ij = C_i^T H C_j over every occupied pair of neighbouring groups: the MOs are     */
/* localized, not canonical, so the whole occupied-occupied block of F enters.  H is   */
/* not truncated here.  Values on the atom-block pattern (the layout of S_val).        */

int orc_gradient(orc_t* o, double* dx_val, double* ds_val) {
  const int G = o->n_groups;
  const int64_t nnz = o->rp[o->n_ao];
  coulomb_q(o);
  double* Hg = xcalloc(nnz, sizeof(double));
  for (int mu = 0; mu < o->n_ao; ++mu) {
    const double qa = o->Q[o->ao_atom[mu]];
    for (int64_t k = o->rp[mu]; k < o->rp[mu + 1]; ++k)
      Hg[k] = o->fock_full ? o->Fuser[k] : o->H0[k] + 0.5 * o->S[k] * (qa + o->Q[o->ao_atom[o->ci[k]]]);
  }
  /* F_ij = C_i^T H C_j, i and j occupied in neighbouring groups; block (g, h) as in O */
  double* F = xcalloc(o->ob_off[o->gn_ptr[G]], sizeof(double));
#pragma omp parallel
  {
    double* y = xcalloc(o->n_ao, sizeof(double));
    uint8_t* mark = xcalloc(o->n_ao, 1);
    int32_t* list = xcalloc(o->n_ao, sizeof(int32_t));
#pragma omp for schedule(dynamic, 4)
    for (int j = 0; j < o->n_occ; ++j) {
      const int32_t nt = spmv_col(o, Hg, &o->C[j], y, mark, list);
      const int h = o->mo_group[j], jl = o->mo_local[j], nh = n_in_group(o, h);
      for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) {
        const int g = o->gn[k];
        const int kk = o->gn_pos[(size_t)g * G + h];
        double* Fgh = F + o->ob_off[o->gn_ptr[g] + kk];
        for (int il = 0; il < n_in_group(o, g); ++il) {
          const int i = o->gm[o->gm_ptr[g] + il];
          if (i >= o->n_occ) break;
          Fgh[(size_t)il * nh + jl] = col_dot_dense(&o->C[i], y);
        }
      }
      clear_touched(y, mark, list, nt);
    }
    free(y); free(mark); free(list);
  }
  /* Z_j = sum_i C_i F_ij (dense column per occupied j, kept as rows of Z) */
  double* Z = xcalloc((size_t)o->n_ao * o->n_occ, sizeof(double));   /* Z[u * n_occ + j] */
#pragma omp parallel for schedule(dynamic, 4)
  for (int j = 0; j < o->n_occ; ++j) {
    const int h = o->mo_group[j], jl = o->mo_local[j], nh = n_in_group(o, h);
    for (int k = o->gn_ptr[h]; k < o->gn_ptr[h + 1]; ++k) {
      const int g = o->gn[k];
      const int kk = o->gn_pos[(size_t)g * G + h];
      const double* Fgh = F + o->ob_off[o->gn_ptr[g] + kk];
      for (int il = 0; il < n_in_group(o, g); ++il) {
        const int i = o->gm[o->gm_ptr[g] + il];
        if (i >= o->n_occ) break;
        const double f = Fgh[(size_t)il * nh + jl];
        for (int32_t t = 0; t < o->C[i].n; ++t) Z[(size_t)o->C[i].row[t] * o->n_occ + j] += o->C[i].val[t] * f;
      }
    }
  }
  /* W_uv = 2 sum_j C_uj Z_vj on the pattern of S (Z is dense, n_ao x n_occ: this
   * reference is meant for systems of a few thousand atoms) */
  double* W = xcalloc(nnz, sizeof(double));
  {
    int64_t* rptr = xcalloc(o->n_ao + 1, sizeof(int64_t));
    for (int j = 0; j < o->n_occ; ++j)
      for (int32_t t = 0; t < o->C[j].n; ++t) rptr[o->C[j].row[t] + 1]++;
    for (int mu = 0; mu < o->n_ao; ++mu) rptr[mu + 1] += rptr[mu];
    int32_t* rmo = xcalloc(rptr[o->n_ao] + 1, sizeof(int32_t));
    double* rval = xcalloc(rptr[o->n_ao] + 1, sizeof(double));
    int64_t* fillp = xcalloc(o->n_ao, sizeof(int64_t));
    for (int j = 0; j < o->n_occ; ++j)
      for (int32_t t = 0; t < o->C[j].n; ++t) {
        const int mu = o->C[j].row[t];
        const int64_t q = rptr[mu] + fillp[mu]++;
        rmo[q] = j; rval[q] = o->C[j].val[t];
      }
    free(fillp);
#pragma omp parallel for schedule(dynamic, 16)
    for (int mu = 0; mu < o->n_ao; ++mu)
      for (int64_t k = o->rp[mu]; k < o->rp[mu + 1]; ++k) {
        const double* zr = Z + (size_t)o->ci[k] * o->n_occ;
        double s = 0.0;
        for (int64_t t = rptr[mu]; t < rptr[mu + 1]; ++t) s += rval[t] * zr[rmo[t]];
        W[k] = 2.0 * s;
      }
    free(rptr); free(rmo); free(rval);
  }
  memset(dx_val, 0, sizeof(double) * o->nblkval);
  memset(ds_val, 0, sizeof(double) * o->nblkval);
  for (int mu = 0; mu < o->n_ao; ++mu) {
    const double qa = o->Q[o->ao_atom[mu]];
    for (int64_t k = o->rp[mu]; k < o->rp[mu + 1]; ++k) {
      const double qb = o->Q[o->ao_atom[o->ci[k]]];
      dx_val[o->ao2blk[k]] = o->P[k];
      ds_val[o->ao2blk[k]] = -W[k] + (o->fock_full ? 0.0 : 0.5 * o->P[k] * (qa + qb));
    }
  }
  free(Hg); free(F); free(Z); free(W);
  return ORC_OK;
}

static int64_t nnz_c(const orc_t* o) {
  int64_t n = 0;
  for (int j = 0; j < o->n_mo; ++j) n += o->C[j].n;
  return n;
}

/* ----------------------------------------------------------------------------------- */
/* public API                                                                          */

void orc_destroy(orc_t* o) {
  if (!o) return;
  trace_clear(o);
  free(o->trace);
  if (o->C) for (int j = 0; j < o->n_mo; ++j) col_free(&o->C[j]);
  void* ptrs[] = {o->atom_nao, o->ao_off, o->ao_atom, o->xyz, o->U, o->q0, o->atom_group,
                  o->blk_rowptr, o->blk_col, o->blk_off, o->rp, o->ci, o->ao2blk, o->S, o->H0,
                  o->H, o->Fuser, o->mo_group, o->mo_local, o->C, o->gm_ptr, o->gm, o->g_nocc,
                  o->gnbr, o->gn_ptr, o->gn, o->gn_pos, o->ob_off, o->O, o->jb_g, o->jb_h,
                  o->jb_round, o->jb_of, o->jb_foff, o->F, o->Fdiag, o->rot_i, o->rot_a,
                  o->rot_blk, o->rot_c, o->rot_s, o->q, o->q_prev, o->dq, o->Q, o->P};
  for (size_t t = 0; t < sizeof(ptrs) / sizeof(ptrs[0]); ++t) free(ptrs[t]);
  free(o);
}

const char* orc_last_error(const orc_t* o) { return o ? o->err : "null oracle"; }

int orc_create(const orc_desc* d, orc_t** out) {
  *out = NULL;
  if (!d || d->n_atoms <= 0 || d->n_mo <= 0 || d->n_occ < 0 || d->n_occ > d->n_mo || d->n_groups <= 0)
    return ORC_E_ARG;
  if (!(d->eps >= 0.0) || !(d->r_nbr_bohr > 0.0)) return ORC_E_ARG;
#ifdef _OPENMP
  if (d->n_threads > 0) omp_set_num_threads(d->n_threads);
#endif
  orc_t* o = calloc(1, sizeof(orc_t));
  *out = o;
  o->criterion = 0; o->step_ortho = 1; o->dq_conv = 0.0;
  o->eps = d->eps; o->e_conv = d->e_conv; o->r_nbr = d->r_nbr_bohr; o->rot_cap_factor = d->rot_cap_factor;
  o->max_sweeps_init = d->max_sweeps_init; o->max_sweeps_step = d->max_sweeps_step; o->scc = d->scc;
  o->n_atoms = d->n_atoms; o->n_mo = d->n_mo; o->n_occ = d->n_occ; o->n_groups = d->n_groups;
  const int na = d->n_atoms;
  o->atom_nao = xcalloc(na, sizeof(int32_t)); memcpy(o->atom_nao, d->atom_nao, na * sizeof(int32_t));
  o->ao_off = xcalloc(na + 1, sizeof(int64_t));
  for (int a = 0; a < na; ++a) o->ao_off[a + 1] = o->ao_off[a] + o->atom_nao[a];
  o->n_ao = (int)o->ao_off[na];
  o->ao_atom = xcalloc(o->n_ao, sizeof(int32_t));
  for (int a = 0; a < na; ++a) for (int64_t mu = o->ao_off[a]; mu < o->ao_off[a + 1]; ++mu) o->ao_atom[mu] = a;
  o->xyz = xcalloc(3 * na, sizeof(double)); memcpy(o->xyz, d->xyz_bohr, 3 * na * sizeof(double));
  o->U = xcalloc(na, sizeof(double)); memcpy(o->U, d->hubbard_u, na * sizeof(double));
  o->q0 = xcalloc(na, sizeof(double)); memcpy(o->q0, d->q0, na * sizeof(double));
  o->atom_group = xcalloc(na, sizeof(int32_t)); memcpy(o->atom_group, d->atom_group, na * sizeof(int32_t));
  for (int a = 0; a < na; ++a)
    if (o->atom_group[a] < 0 || o->atom_group[a] >= o->n_groups || !(o->U[a] > 0.0))
      return fail(o, ORC_E_ARG, "bad atom group or Hubbard parameter");
  o->nblk = d->blk_rowptr[na];
  o->blk_rowptr = xcalloc(na + 1, sizeof(int64_t)); memcpy(o->blk_rowptr, d->blk_rowptr, (na + 1) * sizeof(int64_t));
  o->blk_col = xcalloc(o->nblk, sizeof(int32_t)); memcpy(o->blk_col, d->blk_col, o->nblk * sizeof(int32_t));
  o->blk_off = xcalloc(o->nblk, sizeof(int64_t)); memcpy(o->blk_off, d->blk_off, o->nblk * sizeof(int64_t));
  o->nblkval = 0;
  for (int a = 0; a < na; ++a)
    for (int64_t k = o->blk_rowptr[a]; k < o->blk_rowptr[a + 1]; ++k) {
      const int b = o->blk_col[k];
      if (b < 0 || b >= na || (k > o->blk_rowptr[a] && o->blk_col[k - 1] >= b))
        return fail(o, ORC_E_ARG, "atom-block pattern columns must be sorted and in range");
      const int64_t end = o->blk_off[k] + (int64_t)o->atom_nao[a] * o->atom_nao[b];
      if (end > o->nblkval) o->nblkval = end;
    }
  if (build_ao_csr(o) != ORC_OK) return fail(o, ORC_E_ALLOC, "allocation failed");
  fill_ao_csr(o, d->S_val, d->H0_val);
  for (int64_t k = 0; k < o->rp[o->n_ao]; ++k)
    if (!isfinite(o->S[k]) || !isfinite(o->H0[k])) return fail(o, ORC_E_ARG, "non-finite S or H0");
  if (!check_symmetric(o, o->S) || !check_symmetric(o, o->H0))
    return fail(o, ORC_E_ARG, "S and H0 must be symmetric on a symmetric pattern");
  /* MOs and groups */
  o->mo_group = xcalloc(o->n_mo, sizeof(int32_t)); memcpy(o->mo_group, d->mo_group, o->n_mo * sizeof(int32_t));
  o->gm_ptr = xcalloc(o->n_groups + 1, sizeof(int32_t));
  for (int j = 0; j < o->n_mo; ++j) {
    if (o->mo_group[j] < 0 || o->mo_group[j] >= o->n_groups) return fail(o, ORC_E_ARG, "bad MO group");
    o->gm_ptr[o->mo_group[j] + 1]++;
  }
  for (int g = 0; g < o->n_groups; ++g) o->gm_ptr[g + 1] += o->gm_ptr[g];
  o->gm = xcalloc(o->n_mo, sizeof(int32_t));
  o->mo_local = xcalloc(o->n_mo, sizeof(int32_t));
  o->g_nocc = xcalloc(o->n_groups, sizeof(int32_t));
  {
    int32_t* fillp = xcalloc(o->n_groups, sizeof(int32_t));
    for (int j = 0; j < o->n_mo; ++j) {
      const int g = o->mo_group[j];
      o->mo_local[j] = fillp[g];
      o->gm[o->gm_ptr[g] + fillp[g]++] = j;
      if (j < o->n_occ) o->g_nocc[g]++;
    }
    free(fillp);
  }
  o->C = xcalloc(o->n_mo, sizeof(col_t));
  for (int j = 0; j < o->n_mo; ++j) {
    const int64_t b = d->c0_colptr[j], e = d->c0_colptr[j + 1];
    o->C[j].n = (int32_t)(e - b);
    o->C[j].row = malloc(sizeof(int32_t) * (e > b ? e - b : 1));
    o->C[j].val = malloc(sizeof(double) * (e > b ? e - b : 1));
    for (int64_t t = b; t < e; ++t) {
      if (d->c0_row[t] < 0 || d->c0_row[t] >= o->n_ao || (t > b && d->c0_row[t] <= d->c0_row[t - 1]) ||
          !isfinite(d->c0_val[t]))
        return fail(o, ORC_E_ARG, "C0 rows must be sorted, unique, in range; values finite");
      o->C[j].row[t - b] = d->c0_row[t];
      o->C[j].val[t - b] = d->c0_val[t];
    }
  }
  build_group_nbr(o);
  const int G = o->n_groups;
  o->ob_off = xcalloc(o->gn_ptr[G] + 1, sizeof(int64_t));
  for (int g = 0; g < G; ++g)
    for (int k = o->gn_ptr[g]; k < o->gn_ptr[g + 1]; ++k)
      o->ob_off[k + 1] = o->ob_off[k] + (int64_t)n_in_group(o, g) * n_in_group(o, o->gn[k]);
  o->O = xcalloc(o->ob_off[o->gn_ptr[G]], sizeof(double));
  if (!o->O) return fail(o, ORC_E_ALLOC, "allocation of C^T S C blocks failed");
  build_schedule(o);
  o->Fdiag = xcalloc(o->n_mo, sizeof(double));
  o->q = xcalloc(na, sizeof(double)); o->q_prev = xcalloc(na, sizeof(double));
  o->dq = xcalloc(na, sizeof(double)); o->Q = xcalloc(na, sizeof(double));
  o->P = xcalloc(o->rp[o->n_ao], sizeof(double));
  /* initial orthonormalization (section 3.4) */
  int sweeps = 0, conv = 0;
  double eta = 0.0;
  const double t0 = now_s();
  int rc = orthonormalize(o, 0, o->max_sweeps_init, &sweeps, &eta, &conv);
  if (rc != ORC_OK) return rc;
  if (!conv) return fail(o, ORC_E_ORTHO, "initial orthonormalization did not converge");
  const double t1 = now_s();
  density_charges(o);
  energy(o);
  memcpy(o->q_prev, o->q, na * sizeof(double));
  memset(&o->init_info, 0, sizeof(o->init_info));
  o->init_info.energy = o->E;
  o->init_info.e_band = o->e_band;
  o->init_info.e_coul = o->e_coul;
  o->init_info.ortho_eta = eta;
  o->init_info.n_ortho_sweeps = sweeps;
  o->init_info.ortho_converged = conv;
  o->init_info.nnz_c = nnz_c(o);
  o->init_info.t_ortho = t1 - t0;
  o->init_info.t_charges = now_s() - t1;
  return ORC_OK;
}

int orc_init_info(const orc_t* o, orc_step_info* info) { *info = o->init_info; return ORC_OK; }

int orc_set_fock(orc_t* o, const double* f_val, int32_t mode) {
  if (!f_val || (mode != 0 && mode != 1)) return fail(o, ORC_E_ARG, "bad set_fock arguments");
  for (int64_t k = 0; k < o->nblkval; ++k) if (!isfinite(f_val[k])) return fail(o, ORC_E_ARG, "non-finite Fock");
  if (mode == 0) {
    for (int64_t k = 0; k < o->rp[o->n_ao]; ++k) o->H0[k] = f_val[o->ao2blk[k]];
    if (!check_symmetric(o, o->H0)) return fail(o, ORC_E_ARG, "H0 must be symmetric");
    o->fock_full = 0;
  } else {
    if (!o->Fuser) o->Fuser = xcalloc(o->rp[o->n_ao], sizeof(double));
    for (int64_t k = 0; k < o->rp[o->n_ao]; ++k) o->Fuser[k] = f_val[o->ao2blk[k]];
    if (!check_symmetric(o, o->Fuser)) return fail(o, ORC_E_ARG, "Fock must be symmetric");
    o->fock_full = 1;
  }
  return ORC_OK;
}

int orc_step(orc_t* o, orc_step_info* info) {
  orc_step_info s;
  memset(&s, 0, sizeof(s));
  const double E_prev = o->E;
  if (o->count_on || o->trace_on) work_reset(o);
  double t = now_s(), t2;
  fock_build(o);                                   /* step IV: Fock matrix */
  t2 = now_s(); s.t_fock = t2 - t; t = t2;
  if (o->count_on) {
    work_product(o, o->H, o->n_mo);
    work_fock_blocks(o);
  }
  s.max_abs_fov = fmo(o);                          /* C^T H C */
  t2 = now_s(); s.t_fmo = t2 - t; t = t2;
  s.n_candidates = select_rotations(o);            /* step V */
  s.n_rotations = o->n_rot;
  t2 = now_s(); s.t_select = t2 - t; t = t2;
  apply_rotations(o);
  t2 = now_s(); s.t_rotate = t2 - t; t = t2;
  int sweeps = 0, conv = 0, rc = ORC_OK;
  double eta = 0.0;
  if (o->step_ortho) {
    rc = orthonormalize(o, 0, o->max_sweeps_step, &sweeps, &eta, &conv);  /* step III */
    if (rc != ORC_OK) return rc;
  }
  s.n_ortho_sweeps = sweeps; s.ortho_eta = eta; s.ortho_converged = conv;
  t2 = now_s(); s.t_ortho = t2 - t; t = t2;
  memcpy(o->q_prev, o->q, o->n_atoms * sizeof(double));
  density_charges(o);
  double dqm = 0.0;
  for (int a = 0; a < o->n_atoms; ++a) if (fabs(o->q[a] - o->q_prev[a]) > dqm) dqm = fabs(o->q[a] - o->q_prev[a]);
  s.dq_max = dqm;
  t2 = now_s(); s.t_charges = t2 - t; t = t2;
  energy(o);
  s.delta_e = o->E - E_prev;
  s.converged = o->criterion ? (dqm < o->dq_conv) : (fabs(s.delta_e) < o->e_conv);
  if (s.converged) {
    /* occupied-only orthonormalization after convergence (section 4.1) */
    int sw2 = 0, cv2 = 0;
    double eta2 = 0.0;
    rc = orthonormalize(o, 1, o->max_sweeps_step, &sw2, &eta2, &cv2);
    if (rc != ORC_OK) return rc;
    s.post_ortho = 1;
    density_charges(o);
    energy(o);
  }
  t2 = now_s(); s.t_energy = t2 - t;
  s.energy = o->E; s.e_band = o->e_band; s.e_coul = o->e_coul;
  s.nnz_c = nnz_c(o);
  if (info) *info = s;
  return ORC_OK;
}

int orc_set_literal(orc_t* o, int32_t literal_rot, int32_t literal_ortho) {
  if (!o) return ORC_E_ARG;
  o->literal_rot = literal_rot != 0;
  o->literal_ortho = literal_ortho != 0;
  return ORC_OK;
}

int orc_set_control(orc_t* o, double eps, double e_conv, double dq_conv, int32_t criterion, int32_t step_ortho) {
  if (!(eps >= 0.0) || !isfinite(eps) || !(e_conv >= 0.0) || !(dq_conv >= 0.0) || (criterion != 0 && criterion != 1) ||
      (step_ortho != 0 && step_ortho != 1))
    return fail(o, ORC_E_ARG, "bad control values");
  o->eps = eps; o->e_conv = e_conv; o->dq_conv = dq_conv; o->criterion = criterion; o->step_ortho = step_ortho;
  return ORC_OK;
}

/* step III on demand (section 2): all MOs (restart from improved MOs, e.g. between the
 * loose and the user thresholds of section 4.1) or the occupied ones only; then charges
 * and energy.  Up to max_sweeps_init sweeps; not reaching eps/100 is an error. */
int orc_orthonormalize(orc_t* o, int32_t only_occ, orc_step_info* info) {
  orc_step_info s;
  memset(&s, 0, sizeof(s));
  if (o->count_on || o->trace_on) work_reset(o);
  int sweeps = 0, conv = 0;
  double eta = 0.0;
  int rc = orthonormalize(o, only_occ ? 1 : 0, o->max_sweeps_init, &sweeps, &eta, &conv);
  if (rc != ORC_OK) return rc;
  if (!conv) return fail(o, ORC_E_ORTHO, "orthonormalization did not converge");
  density_charges(o);
  energy(o);
  s.energy = o->E; s.e_band = o->e_band; s.e_coul = o->e_coul;
  s.n_ortho_sweeps = sweeps; s.ortho_eta = eta; s.ortho_converged = conv; s.nnz_c = nnz_c(o);
  if (info) *info = s;
  return ORC_OK;
}

double orc_energy(const orc_t* o) { return o->E; }

int orc_density(const orc_t* o, double* p_val) {
  memset(p_val, 0, sizeof(double) * o->nblkval);
  for (int64_t k = 0; k < o->rp[o->n_ao]; ++k) p_val[o->ao2blk[k]] = o->P[k];
  return ORC_OK;
}

int orc_charges(const orc_t* o, double* q) { memcpy(q, o->q, sizeof(double) * o->n_atoms); return ORC_OK; }

int64_t orc_nnz_c(const orc_t* o) { return nnz_c(o); }

int orc_get_c(const orc_t* o, int64_t* colptr, int32_t* row, double* val, int64_t cap) {
  if (nnz_c(o) > cap) return -1;
  colptr[0] = 0;
  for (int j = 0; j < o->n_mo; ++j) {
    memcpy(row + colptr[j], o->C[j].row, sizeof(int32_t) * o->C[j].n);
    memcpy(val + colptr[j], o->C[j].val, sizeof(double) * o->C[j].n);
    colptr[j + 1] = colptr[j] + o->C[j].n;
  }
  return 0;
}

int orc_n_blocks(const orc_t* o) { return o->n_blocks; }

int orc_schedule(const orc_t* o, int32_t* g, int32_t* h, int32_t* round) {
  for (int b = 0; b < o->n_blocks; ++b) { g[b] = o->jb_g[b]; h[b] = o->jb_h[b]; round[b] = o->jb_round[b]; }
  return o->n_rounds;
}

int orc_group_nbr(const orc_t* o, uint8_t* out) {
  memcpy(out, o->gnbr, (size_t)o->n_groups * o->n_groups);
  return 0;
}

int orc_fdiag(const orc_t* o, double* out) { memcpy(out, o->Fdiag, sizeof(double) * o->n_mo); return 0; }
int orc_n_rot(const orc_t* o) { return o->n_rot; }
int orc_rotations(const orc_t* o, int32_t* i, int32_t* a, double* c, double* s) {
  for (int t = 0; t < o->n_rot; ++t) { i[t] = o->rot_i[t]; a[t] = o->rot_a[t]; c[t] = o->rot_c[t]; s[t] = o->rot_s[t]; }
  return o->n_rot;
}

/* ---- measurement only ---------------------------------------------------------------- */

int orc_set_count(orc_t* o, int32_t on) { o->count_on = on != 0; return ORC_OK; }
int orc_work_get(const orc_t* o, orc_work* out) { *out = o->work; return ORC_OK; }
int orc_set_trace(orc_t* o, int32_t on) { o->trace_on = on != 0; return ORC_OK; }
int orc_trace_sweeps(const orc_t* o) { return o->n_trace; }

int orc_trace_sizes(const orc_t* o, int32_t k, int32_t* n_scope, int64_t* nnz, int64_t* n_sel, double* eta) {
  if (k < 0 || k >= o->n_trace) return ORC_E_ARG;
  const struct trace_sweep* t = &o->trace[k];
  *n_scope = t->n_scope; *nnz = t->nnz; *n_sel = t->n_sel; *eta = t->eta;
  return ORC_OK;
}

int orc_trace_get(const orc_t* o, int32_t k, int64_t* colptr, int32_t* row, double* val, int32_t* sel_i,
                  int32_t* sel_j, double* sel_d) {
  if (k < 0 || k >= o->n_trace) return ORC_E_ARG;
  const struct trace_sweep* t = &o->trace[k];
  memcpy(colptr, t->colptr, sizeof(int64_t) * (t->n_scope + 1));
  memcpy(row, t->row, sizeof(int32_t) * t->nnz);
  memcpy(val, t->val, sizeof(double) * t->nnz);
  memcpy(sel_i, t->si, sizeof(int32_t) * t->n_sel);
  memcpy(sel_j, t->sj, sizeof(int32_t) * t->n_sel);
  memcpy(sel_d, t->sd, sizeof(double) * t->n_sel);
  return ORC_OK;
}

int orc_fov(const orc_t* o, double* out, int64_t* n) {
  *n = o->jb_foff[o->n_blocks];
  if (out) memcpy(out, o->F, sizeof(double) * (size_t)*n);
  return ORC_OK;
}

int orc_fock(const orc_t* o, double* out) {
  memset(out, 0, sizeof(double) * o->nblkval);
  for (int64_t k = 0; k < o->rp[o->n_ao]; ++k) out[o->ao2blk[k]] = o->H[k];
  return ORC_OK;
}
