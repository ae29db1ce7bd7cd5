// Internal declarations of the gfx950 sparse SCF library: data layout and
// kernel launchers.  Not part of the public C ABI (include/sscf.h).
//
// Layout in HBM (MI355X, 288 GB per GPU):
//  * AOs are grouped in row blocks of RB = 16 consecutive AOs (n_rb blocks).
//  * The MOs of MO group g (section 3.2) form panel g of W columns: occupied
//    MOs in columns [0, OW), virtual MOs in [OW, OW + VW) = [OW, W); unused
//    columns are zero.  W, OW, VW are multiples of 16.
//  * C is stored as a pool of tiles: tile (g, r) holds rows 16 r .. 16 r + 15 of
//    panel g as a row-major 16 x W block at C + slot[g * n_rb + r] * 16 W; the slot
//    table gives every tile a slot (dense capacity) or only those near the group.
//    act[g * n_rb + r] tells whether the tile may hold nonzeros; an inactive C
//    tile is all zeros.  list[g * n_rb + t], t < cnt[g], are the active row
//    blocks of panel g in increasing order.
//  * S, H0 and H are stored as 16 x 16 row-major blocks on the row-block
//    pattern of the atom-neighbour map (block-CSR: xs_ptr, xs_col, xs_row).
//  * C^T S C is kept as W x W blocks for the unordered neighbour pairs
//    (g <= h); the occupied-virtual part of C^T H C as OW x VW blocks for the
//    Jacobi blocks (g occupied, h virtual).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sscf {

constexpr int RB = 16;           // AOs per row block
// strided parts of the split reductions (column dot products; Coulomb sums over atoms)
constexpr int CD_SPLIT = 16, CL_SPLIT = 16;
constexpr int ZERO_DOUBLES = 128 * 64;  // zero buffer of the kernels' masked loads (64 KB)
constexpr int GUESS_MAXN = 8;            // AOs of the largest fragment of the initial guess
constexpr int MAX_W = 128;       // widest panel supported
constexpr int KM_SLOTS = 2048;         // LDS candidates of one mean in a k-means round
constexpr int KM_MAX_LINK = 1024;      // largest n_link (a chunk scans KM_SLOTS - n_link points)
constexpr int KM_MAX_MEANS = 4096;     // most means (the per-point sort of means lives in LDS)
constexpr int KM_PCAP = 256;           // proposals listed per mean and round (more: a scan of all points)
static_assert(KM_MAX_LINK + KM_PCAP <= KM_SLOTS, "listed proposals and kept points must fit in the LDS slots");
constexpr int MAX_TIES = 4096;
constexpr int NB_TILE_ATOMS = 64;       // atoms per tile of the atom neighbour map   // candidates sharing the cut-off |F| that can be ordered

// scalars shared between kernels and the host (one device copy per context)
struct Scalars {
  unsigned long long eta_bits;      // max |D_ij| (bits of a non-negative double)
  unsigned long long fov_bits;      // max |F_ia|
  unsigned long long dq_bits;       // max |q_a - q_prev_a|
  unsigned long long cut_key;       // |F| key of the last selected rotation
  long long tie_cut;                // largest (i * n_mo + a) taken among ties at cut_key
  long long remaining;              // radix selection state
  unsigned long long prefix, mask;
  int n_cand;
  int n_rot;
  int err;                          // 1: non-positive diagonal of C^T S C
  int tie_count;                    // keys equal to cut_key (from the last radix pass)
  int tie_n;                        // tie keys collected
  double e_band, e_coul;
  double eta;
  int cap_err;                      // 1 + the first tile where a nonzero fell without a slot (sticky)
};

struct View {
  // sizes
  int n_atoms, n_ao, n_rb, n_mo, n_occ, G, W, OW, VW;
  // geometry
  const double* xyz;
  const double* U;
  const double* q0;
  const int* ao_atom;
  // row-block pattern
  int nbx;
  const int* xs_ptr;
  const int* xs_col;
  const int* xs_row;
  // ZERO_DOUBLES zero doubles: the target of loads that are known to give zero
  const double* zeros;
  // tile capacity: slot[g * n_rb + r] is the slot of tile (g, r) in the pools of C and its FP32
  // copy (n_slots tiles of 16 x W each), -1 when the tile has no slot (then it is zero and must
  // stay so: a nonzero landing there records the tile in *cap_err).  slotY does the same for the products
  // Y = X C (and what shares their pools): its tiles are the row blocks that X's pattern links
  // to a tile of C with a slot, so a product never falls outside it.
  const int* slot;
  const int* slotY;
  int max_c, max_y;   // the most tiles with a slot in any one group (C, Y): bounds a panel's lists
  int* cap_err;
};

// ---- launchers (sscf_kernels.hip) ------------------------------------------------------
void launch_fill(double* p, size_t n, double v, hipStream_t s);
void launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t s);
void launch_fill_i32(int* p, size_t n, int v, hipStream_t s);
void launch_scatter_c0(const View& v, int nnz, const int64_t* colptr_expanded_col, const int* row,
                       const double* val, const int* mo_panel, const int* mo_col, double* C,
                       uint8_t* act, unsigned int* cmask, int* cap_err, hipStream_t s);
// actY = the row blocks that S links to a tile of the lists listC / cntC (the lists of the
// current activity flags), scattered through the symmetric pattern of S
void launch_dilate(const View& v, const int* listC, const int* cntC, uint8_t* actY, hipStream_t s);
void launch_list(const View& v, const uint8_t* act, int* list, int* cnt, hipStream_t s);
// per row block, the groups active there (ascending): listT[r G + k], k < cntT[r]
void launch_list_t(const View& v, const uint8_t* act, int* listT, int* cntT, hipStream_t s);
void launch_spmm(const View& v, const double* X, const double* C, const uint8_t* actC,
                 const unsigned int* cmask, const int* listY, const int* cntY, double* Y,
                 unsigned int* ymask, unsigned int smask, unsigned long long* ctr, hipStream_t s);
// perm / maxc: the items of a list sorted by group, laid out per XCD (see xcd_perm)
void launch_pair(const View& v, int n_pairs, const int* perm, int maxc, const int* pg, const int* ph, const double* C,
                 const int* listC, const int* cntC, const unsigned int* cmask, const double* Y,
                 const uint8_t* actY, const unsigned int* ymask, int row_off, int MT, int col_off,
                 int NT, double* out, int ld, size_t out_stride, unsigned long long* ctr,
                 hipStream_t s);
void launch_coldot(const View& v, const double* C, const int* listC, const int* cntC, const unsigned int* cmask,
                   const double* Y, const uint8_t* actY, double* part, double* out, hipStream_t s);
void launch_ortho_scale(const View& v, int n_pairs_self, const int* self_pair, const double* O,
                        const int* pnocc, const int* pnvirt, int occ_only, double* sc,
                        Scalars* sd, hipStream_t s);
void launch_normalize_d(const View& v, int n_pairs, const int* pg, const int* ph, double* O,
                        double* Dt, const double* sc, const int* pnocc, const int* pnvirt,
                        int occ_only, Scalars* sd, hipStream_t s);
void launch_scale_c(const View& v, double* C, const int* listC, const int* cntC, const unsigned int* cmask,
                    const double* sc, hipStream_t s);
void launch_mark_selected(const View& v, int n_pairs, const int* pg, const int* ph, const double* D,
                          const Scalars* sd, uint8_t* pair_sel, uint8_t* upd, uint8_t* rmask, int* nsel,
                          hipStream_t s);
// act_new = support of C after the combinations of the selected pairs.  With mask, only the tiles
// where mask is set (no capacity test); without, a tile with no slot is marked 2 (a tile the
// combination computes only to check that it stays zero).
void launch_update_support(const View& v, const int* listC, const int* cntC, int n_pairs, const int* pg,
                           const int* ph, const uint8_t* pair_sel, const uint8_t* mask, uint8_t* act_new,
                           hipStream_t s);
void launch_clear_flags(const View& v, uint8_t* act, unsigned int* cmask, const int* list, const int* cnt,
                        hipStream_t s);
void launch_tile_flags(const View& v, const double* C, const int* list, const int* cnt, uint8_t* act,
                       unsigned int* cmask, ulonglong2* colm, hipStream_t s);
// sc: the sweep's column norms; the packed columns are C's divided by them
void launch_pack_cols(const View& v, const double* C, const int* list, const int* cnt, int col_end,
                      const double* sc, double* P, uint8_t* cidx, uint8_t* ncol, hipStream_t s);
void launch_ortho_update(const View& v, const double* C, const uint8_t* actC, const unsigned int* cmaskC,
                         const double* P, const uint8_t* cidx,
                         const uint8_t* ncol, const int* gn_ptr, const int* gn, const int* pair_of,
                         const uint8_t* pair_sel, const double* D, const double* Dt, const uint8_t* rmask,
                         const Scalars* sd, const uint8_t* upd, const double* sc, double cut, const int* listN,
                         const int* cntN, double* Cn, uint8_t* actN, unsigned int* cmaskN, unsigned long long* ctr,
                         hipStream_t s);
void launch_coulomb(const View& v, int scc, const double* dq, double* part, double* Q, hipStream_t s);
void launch_fock(const View& v, const double* S, const double* H0, const double* Hfull,
                 const double* Q, double eps, double* H, float* H32, hipStream_t s);
void launch_count_candidates(int nb, int OW, int VW, const int* jb_nocc, const int* jb_nvirt,
                             const double* F, double tau, Scalars* sd, hipStream_t s);
void launch_radix_pass(int nb, int OW, int VW, const int* jb_nocc, const int* jb_nvirt,
                       const double* F, double tau, int shift, Scalars* sd, unsigned int* hist,
                       hipStream_t s);
void launch_sel_init(Scalars* sd, long long K, int select_all, hipStream_t s);
void launch_sel_finish(Scalars* sd, hipStream_t s);
void launch_tie_cut(int nb, int OW, int VW, const int* jb_g, const int* jb_h, const int* jb_nocc,
                    const int* jb_nvirt, const double* F, const int* mo_of, int W, long long n_mo,
                    double tau, Scalars* sd, long long* ties, hipStream_t s);
void launch_block_select(const View& v, int nb, const int* jb_g, const int* jb_h, const int* jb_nocc,
                         const int* jb_nvirt, const double* F, const double* Fdiag, const int* mo_of,
                         double tau, Scalars* sd, int* rot_cnt, int2* rot_slot, double2* rot_cs,
                         int* tcnt, int* tcol, ulonglong2* tmask, int fp32, hipStream_t s);
void launch_compose_rot(const View& v, int nb, const int* rot_cnt, const int2* rot_slot,
                        const double2* rot_cs, const int* tcnt, double* R, float* R32, hipStream_t s);
void launch_round_meta(int n_rounds, const int* round_ptr, const int* round_list, const int* rot_cnt,
                       const int* jb_g, const int* jb_h, const int* tcnt, int* rcnt, int* roff, int4* meta,
                       hipStream_t s);
void launch_group_nbr(int n_atoms, int G, const double* xyz, const int* atom_group, const int* ga_ptr, const int* ga,
                      double r_nbr, uint8_t* gnbr, hipStream_t s);
void launch_fragment_guess(int n_frag, const int* frag_atom0, const int64_t* ao_off, const int64_t* blk_rowptr,
                           const int* blk_col, const int64_t* blk_off, const int* atom_nao, const double* S,
                           const double* H, const int64_t* frag_coff, double* out, double* lam, int* err,
                           hipStream_t s);
void launch_check_coords(int64_t n, const double* x, int* flag, hipStream_t s);
void launch_atom_nbr_count(int n, const double* xyz, double cutoff, double* box, int* cnt, int64_t* rowptr,
                           hipStream_t s);
void launch_atom_nbr_fill(int n, const double* xyz, double cutoff, const double* box, const int64_t* rowptr, int* col,
                          hipStream_t s);
void launch_km_rank(int n, int m, const double* pts, const double* means, int* rank, hipStream_t s);
void launch_km_reset(int n, int m, int* assign, int* next, int* n_held, int* pcnt, hipStream_t s);
void launch_km_round(int n, int m, int n_link, const double* pts, const double* means, const int* rank, int* assign,
                     int* next, int* prop, int* pcnt, int* plist, int* held, int* n_held, int* n_free,
                     hipStream_t s);
void launch_km_move(int n, int m, const double* pts, const int* assign, const double* means, double* out,
                    double* disp, hipStream_t s);
void launch_givens_rb(const View& v, int n_rounds, const int* roff, const int4* meta, const ulonglong2* tmask,
                      const int* tcol, const double* R, const float* R32, double eps, double* C, uint8_t* actC,
                      unsigned int* cmask, ulonglong2* colm, const int* rot_cnt, unsigned long long* wcnt,
                      hipStream_t s);
void launch_spmm32(const View& v, const float* X, const float* C, const uint8_t* actC,
                   const unsigned int* cmask, const int* listY, const int* cntY, float* Y,
                   unsigned int* ymask, unsigned long long* ctr, hipStream_t s);
void launch_pair32(const View& v, int n_pairs, const int* perm, int maxc, const int* pg, const int* ph, const float* C,
                   const int* listC, const int* cntC, const unsigned int* cmask, const float* Y,
                   const uint8_t* actY, const unsigned int* ymask, int row_off, int MT, int col_off,
                   int NT, double* out, int ld, size_t out_stride, unsigned long long* ctr,
                   hipStream_t s);
void launch_round_c32(const View& v, const double* C, const int* list, const int* cnt, const unsigned int* cmask,
                      float* C32, hipStream_t s);
void launch_coldot32(const View& v, const float* C, const int* listC, const int* cntC, const unsigned int* cmask,
                     const float* Y, const uint8_t* actY, double* out, hipStream_t s);
void launch_charges_rows(const View& v, const double* C, const int* listTC, const int* cntTC, const double* Y,
                         const uint8_t* actY, const double* sc, const int* pnocc, double* rowq, hipStream_t s);
void launch_atom_charges(const View& v, const int64_t* ao_off, const double* rowq, double* q,
                         double* q_prev, double* dq, Scalars* sd, int shift_prev, hipStream_t s);
void launch_sum_band(const View& v, const double* d, const int* pnocc, Scalars* sd, hipStream_t s);
void launch_sum_coul(const View& v, int scc, const double* dq, const double* Q, Scalars* sd,
                     hipStream_t s);
// listTA/cntTA: launch_list_t of A's activity; cmA / cmB: the 16-column slice masks of A's and
// B's tiles (cmB may be NULL: B's slices not tracked); B_is_y: B lives in the pool of Y (slotY),
// else in that of C
void launch_density_blocks(const View& v, const double* A, const unsigned int* cmA, const int* listTA,
                           const int* cntTA, const double* B, const uint8_t* actB, const unsigned int* cmB,
                           bool B_is_y, double* P, hipStream_t s);
void launch_grad_assemble(const View& v, int64_t n_val, const int64_t* map, const double* P, const double* Wb,
                          const double* Q, int qterm, double* dX, double* dS, hipStream_t s);
void launch_grad_onsite(const View& v, const int64_t* ao_off, const int* xs_diag, const double* P, double* out,
                        hipStream_t s);
void launch_apply_occ(const View& v, const double* C, const uint8_t* actC, const unsigned int* cmask,
                      const int* gn_ptr, const int* gn,
                      const int* pair_of, const int* pg, const double* FA, const double* FB, const int* listZ,
                      const int* cntZ, double* Z, hipStream_t s);
// ---- work counting (sscf_count.hip) --------------------------------------------------------
void launch_cnt_xrow(const View& v, const void* X, bool fp32, int* xrow, unsigned long long* tot, hipStream_t s);
// is_y: T lives in the pool of Y (slotY), else in that of C
void launch_cnt_tiles(const View& v, const void* T, bool fp32, bool is_y, const int* list, const int* cnt, int c0,
                      int c1, const int* weight, int* colnnz, unsigned long long* nnz, unsigned long long* wsum,
                      hipStream_t s);
void launch_row_masks(const View& v, const void* T, bool fp32, bool is_y, const int* list, const int* cnt,
                      ulonglong2* masks, hipStream_t s);
void launch_cnt_pairs(const View& v, int n_items, const int* ig, const int* ih, const int* listC, const int* cntC,
                      const uint8_t* actY, const ulonglong2* mC, const ulonglong2* mY, int a0, int a1, int b0,
                      int b1, int tri, unsigned long long* out, hipStream_t s);
void launch_cnt_dot(size_t n, const int* a, const int* b, unsigned long long* dot, unsigned long long* sumb,
                    hipStream_t s);
void launch_gather(const int64_t* map, int64_t n, const double* src, double* dst, hipStream_t s);
void launch_scatter(const int64_t* map, int64_t n, const double* src, double* dst, hipStream_t s);

}  // namespace sscf
