// Host side of the gfx950 sparse SCF library: the C ABI of include/sscf.h,
// set-up of the patterns and schedules, and the per-step driver.
//
// Paper: A. Scemama, N. Renon, M. Rapacioli, "A Sparse SCF algorithm and its
// parallel implementation: Application to DFTB", arXiv:1402.2880.
//
// Readings of points the paper leaves open (the same ones the test oracle uses):
//  * orthonormalization (section 3.4): each sweep recomputes C^T S C, normalizes,
//    tests max |D_ij| < eps/100 on the normalized matrix D, and otherwise
//    combines every pair with |D_ij| >= 1e-3 max|D| at once, C <- C - 1/2 C D_sel,
//    then zeroes |C| < 1e-3 eps in the combined columns (section 4.1);
//  * partial diagonalization (section 3.5): at most rot_cap_factor * n_occ
//    rotations per step, chosen by decreasing |F_ia| >= eps (ties by (i, a)),
//    applied block round by block round with angles from the F of the start of
//    the step; the rotation is C'_i = c C_i + s C_a, C'_a = -s C_i + c C_a; after
//    each block the rotated columns lose |C| < eps (section 4.1);
//  * each step ends with a full re-orthonormalization; once |dE| < e_conv the
//    occupied MOs are orthonormalized among themselves (section 4.1);
//  * E = sum_uv P_uv H0_uv + 1/2 dq^T gamma dq, P = 2 C_occ C_occ^T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sscf.h"
#include "sscf_internal.h"

using namespace sscf;

namespace {

thread_local std::string g_init_error;

struct Fail {
  sscf_status code;
  std::string msg;
};

[[noreturn]] void fail(sscf_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Fail{code, buf};
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(SSCF_E_HIP, "%s: %s", what, hipGetErrorString(e));
}
#define HIPC(x) hip_check((x), #x)

int round16(int x) { return ((x + 15) / 16) * 16; }

// kernel classes reported by sscf_get_kernel_stats
enum { KC_SPMM, KC_PAIR_O, KC_PAIR_F, KC_UPDATE, KC_GIVENS, KC_SELECT, KC_FOCK };
const char* const KC_NAME[SSCF_N_KERNEL_CLASSES] = {
    "spmm_tiles", "pair_overlap", "pair_fock", "ortho_update", "rotations", "select", "fock"};
// executed FP64/FP32 16 x 16 x 4 matrix-core products: 2048 flops each
const double KC_FLOP_PER_MFMA = 2048.0;

}  // namespace

struct sscf_ctx {
  // parameters
  double eps = 0, e_conv = 0, r_nbr = 0, rot_cap = 0;
  double dq_conv = 0;                   // charge criterion (section 4.1)
  int criterion = SSCF_CONV_ENERGY, step_ortho = 1;
  int max_sweeps_init = 0, max_sweeps_step = 0, scc = 1, precision = 0;
  int fock_full = 0;
  hipStream_t stream = nullptr;
  sscf_allocator alloc{};
  std::vector<void*> owned;
  std::vector<size_t> owned_bytes;
  std::string err;
  bool failed = false;

  // sizes
  View v{};
  int64_t n_val = 0;
  int n_pairs = 0, n_blocks = 0, n_rounds = 0;
  int *pair_perm = nullptr, *jb_perm = nullptr;   // pairs / Jacobi blocks laid out per XCD
  int pair_maxc = 0, jb_maxc = 0;

  // host copies needed after set-up
  std::vector<int> h_pg, h_ph;        // unordered neighbour pairs g <= h
  std::vector<int64_t> h_blk_rowptr, h_blk_off;
  std::vector<int32_t> h_blk_col, h_atom_nao;
  std::vector<int32_t> h_mo_of;      // [G * W] MO index of a panel column, -1 if none
  std::vector<int32_t> h_pnocc, h_pnvirt;
  std::vector<int32_t> h_jb_g, h_jb_h, h_jb_round;
  std::vector<int32_t> h_round_ptr;  // blocks of round r: round_list[round_ptr[r] .. round_ptr[r+1])
  std::vector<int64_t> h_ao_off;

  // device arrays
  double *xyz = nullptr, *U = nullptr, *q0 = nullptr;
  int* ao_atom = nullptr;
  int64_t* ao_off = nullptr;
  int *xs_ptr = nullptr, *xs_col = nullptr, *xs_row = nullptr;
  int* xs_diag = nullptr;            // index of the diagonal block (r, r) of each row block
  int64_t* val_map = nullptr;        // atom-block value index -> row-block element index
  double *S = nullptr, *H0 = nullptr, *H = nullptr, *Hfull = nullptr;
  double* C[2] = {nullptr, nullptr};
  uint8_t* actC[2] = {nullptr, nullptr};
  int* listC[2] = {nullptr, nullptr};
  int* cntC[2] = {nullptr, nullptr};
  unsigned int* cmask[2] = {nullptr, nullptr};   // per tile: 16-column slices that may be nonzero
  int cur = 0;                        // C[cur] is the current MO matrix
  double* Y = nullptr;
  uint8_t* actY = nullptr;
  unsigned int* ymask = nullptr;
  int *listY = nullptr, *cntY = nullptr;
  uint8_t* act_tmp = nullptr;
  int *listT = nullptr, *cntT = nullptr;   // per row block, the groups active in C there
  int *list_tmp = nullptr, *cnt_tmp = nullptr;
  int *pnocc = nullptr, *pnvirt = nullptr, *mo_of = nullptr;
  int *gn_ptr = nullptr, *gn = nullptr, *pair_of = nullptr, *pg = nullptr, *ph = nullptr, *self_pair = nullptr;
  double* O = nullptr;
  double* Dt = nullptr;                 // transposes of the off-diagonal D blocks
  double* sc = nullptr;
  uint8_t *upd = nullptr, *pair_sel = nullptr;
  uint8_t* rmask = nullptr;             // per pair and orientation: selected 16-column slices of each D row
  uint8_t *pcidx = nullptr, *pncol = nullptr;   // packed nonzero columns of the C tiles (values in Y)
  double* part = nullptr;               // partial sums of the split reductions (coldot, coulomb)
  // energy gradient (allocated on first use)
  double *foo_a = nullptr, *foo_b = nullptr, *wblk = nullptr;
  double *gx = nullptr, *gs = nullptr;  // device copies for the host-buffer gradient call
  uint8_t* pair_all = nullptr;        // per pair: nonzero-fragment masks of D_sel and its transpose
  int *jb_g = nullptr, *jb_h = nullptr, *jb_nocc = nullptr, *jb_nvirt = nullptr, *round_list = nullptr;
  double *F = nullptr, *Fdiag = nullptr, *dvec = nullptr;
  int *rot_cnt = nullptr, *tcnt = nullptr, *tcol = nullptr, *round_ptr = nullptr;
  ulonglong2* tmask = nullptr;          // per Jacobi block: its touched panel columns
  ulonglong2* colm = nullptr;           // per tile: nonzero columns (exact during the rotation pass)
  int* slot = nullptr;                  // tile -> slot of the pools of C (-1: none)
  int* slotY = nullptr;                 // tile -> slot of the pools of Y (-1: none)
  size_t n_slots = 0, n_slots_y = 0;
  std::vector<double> cap_gap_g, cap_gap_r, cap_R;   // spheres and radius of each group (report)
  int *rcnt = nullptr, *roff = nullptr;
  int4* rmeta = nullptr;                // blocks with rotations, packed in round order
  int2* rot_slot = nullptr;
  double* Rrot = nullptr;               // composed rotation of each Jacobi block, W x W
  // FP32 form: H, H C and the composed rotations in single precision
  float *H32 = nullptr, *Y32 = nullptr, *R32 = nullptr, *C32 = nullptr;
  double2* rot_cs = nullptr;
  unsigned int* hist = nullptr;
  long long* ties = nullptr;
  double *q = nullptr, *q_prev = nullptr, *dq = nullptr, *Q = nullptr, *rowq = nullptr, *pblk = nullptr,
         *pval = nullptr;
  Scalars* sd = nullptr;
  hipEvent_t ev[8] = {};

  // state
  double E = 0.0;
  sscf_step_info init_info{};

  // optional profiling (SSCF_FLAG_PROFILE): HIP events around the launches of each
  // kernel class, device counters of MFMA tile products / algorithmic bytes
  bool prof = false;
  std::vector<hipEvent_t> pev;
  std::vector<int> pcls;
  int pused = 0;
  double pms[SSCF_N_KERNEL_CLASSES] = {};
  long long plaunch[SSCF_N_KERNEL_CLASSES] = {};
  unsigned long long* pctr = nullptr;

  // optional work counting (SSCF_FLAG_COUNT_WORK): the algorithmic flops and bytes of each
  // pass, counted on the current state by the kernels of sscf_count.hip between the passes
  bool count = false, counting = false;     // counting: inside a step, set-up or step III call
  double wfl[SSCF_N_KERNEL_CLASSES] = {}, wby[SSCF_N_KERNEL_CLASSES] = {};
  unsigned long long* wdev = nullptr;       // 8 scratch counters
  int *w_xrow = nullptr, *w_colnnz = nullptr, *w_nsel = nullptr;
  ulonglong2 *w_mC = nullptr, *w_mY = nullptr;
  bool wc() const { return count && counting; }
  void wzero() { HIPC(hipMemsetAsync(wdev, 0, 8 * sizeof(unsigned long long), stream)); }
  std::array<unsigned long long, 8> wread() {
    std::array<unsigned long long, 8> h{};
    HIPC(hipMemcpyAsync(h.data(), wdev, sizeof(h), hipMemcpyDeviceToHost, stream));
    sync();
    return h;
  }
  // Y = X C over the columns [0, c1) of every panel (X, C, Y in FP32 when fp32)
  void count_product(const void* X, const void* Cp, const void* Yp, bool fp32, bool occ_only) {
    const int c1 = occ_only ? v.OW : v.W;
    wzero();
    launch_fill_i32(w_xrow, (size_t)v.n_rb * RB, 0, stream);
    launch_cnt_xrow(v, X, fp32, w_xrow, wdev + 0, stream);
    launch_cnt_tiles(v, Cp, fp32, false, listC[cur], cntC[cur], 0, c1, w_xrow, nullptr, wdev + 1, wdev + 2, stream);
    launch_cnt_tiles(v, Yp, fp32, true, listY, cntY, 0, c1, nullptr, nullptr, wdev + 3, nullptr, stream);
    const auto w = wread();
    wfl[KC_SPMM] += 2.0 * (double)w[2];
    wby[KC_SPMM] += (fp32 ? 4.0 : 8.0) * ((double)w[0] + (double)w[1] + (double)w[3]);
  }
  // C_g^T Y_h over the items (g, h): columns [a0, a1) of g against [b0, b1) of h
  void count_pairs(int cls, int n_items, const int* ig, const int* ih, const void* Cp, const void* Yp, bool fp32,
                   int a0, int a1, int b0, int b1, int tri, double n_out) {
    wzero();
    launch_row_masks(v, Cp, fp32, false, listC[cur], cntC[cur], w_mC, stream);
    launch_row_masks(v, Yp, fp32, true, listY, cntY, w_mY, stream);
    launch_cnt_pairs(v, n_items, ig, ih, listC[cur], cntC[cur], actY, w_mC, w_mY, a0, a1, b0, b1, tri, wdev + 0,
                     stream);
    launch_cnt_tiles(v, Cp, fp32, false, listC[cur], cntC[cur], a0, a1, nullptr, nullptr, wdev + 1, nullptr, stream);
    launch_cnt_tiles(v, Yp, fp32, true, listY, cntY, b0, b1, nullptr, nullptr, wdev + 2, nullptr, stream);
    const auto w = wread();
    wfl[cls] += 2.0 * (double)w[0];
    wby[cls] += (fp32 ? 4.0 : 8.0) * ((double)w[1] + (double)w[2]) + 8.0 * n_out;   // outputs are FP64
  }
  // unordered MO pairs of C^T S C in scope: i of the lower group, i <= j inside a group
  double overlap_pairs(bool occ_only) const {
    double n = 0.0;
    for (size_t p = 0; p < h_pg.size(); ++p) {
      const double ng = h_pnocc[h_pg[p]] + (occ_only ? 0 : h_pnvirt[h_pg[p]]);
      const double nh = h_pnocc[h_ph[p]] + (occ_only ? 0 : h_pnvirt[h_ph[p]]);
      n += (h_pg[p] == h_ph[p]) ? ng * (ng + 1.0) / 2.0 : ng * nh;
    }
    return n;
  }
  double fock_pairs() const {
    double n = 0.0;
    for (int b = 0; b < n_blocks; ++b) n += (double)h_pnocc[h_jb_g[b]] * (double)h_pnvirt[h_jb_h[b]];
    return n;
  }
  // the combination: 2 nnz(C_i) per selected (i, j); C read, D_sel read (nsel from the marking)
  void count_update_begin(bool occ_only) {
    const int c1 = occ_only ? v.OW : v.W;
    wzero();
    launch_fill_i32(w_colnnz, (size_t)v.G * v.W, 0, stream);
    launch_cnt_tiles(v, C[cur], false, false, listC[cur], cntC[cur], 0, c1, nullptr, w_colnnz, wdev + 0, nullptr, stream);
    launch_cnt_dot((size_t)v.G * v.W, w_colnnz, w_nsel, wdev + 1, wdev + 2, stream);
    const auto w = wread();
    wfl[KC_UPDATE] += 2.0 * (double)w[1];
    wby[KC_UPDATE] += 8.0 * ((double)w[0] + (double)w[2]);
  }
  void count_update_end(int b, bool occ_only) {          // C written: buffer b, listed
    wzero();
    launch_cnt_tiles(v, C[b], false, false, listC[b], cntC[b], 0, occ_only ? v.OW : v.W, nullptr, nullptr, wdev + 0, nullptr,
                     stream);
    wby[KC_UPDATE] += 8.0 * (double)wread()[0];
  }
  int64_t count_nnz_c() {
    wzero();
    launch_cnt_tiles(v, C[cur], false, false, listC[cur], cntC[cur], 0, v.W, nullptr, nullptr, wdev + 0, nullptr, stream);
    return (int64_t)wread()[0];
  }

  int pbegin(int c) {
    if (!prof) return -1;
    if ((size_t)(2 * pused + 2) > pev.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        HIPC(hipEventCreate(&e));
        pev.push_back(e);
      }
    }
    if ((size_t)pused >= pcls.size()) pcls.resize(pused + 32);
    HIPC(hipEventRecord(pev[2 * pused], stream));
    pcls[pused] = c;
    return pused++;
  }
  void pend(int i) {
    if (i >= 0) HIPC(hipEventRecord(pev[2 * i + 1], stream));
  }
  unsigned long long* ctr(int c) { return prof ? pctr + c : nullptr; }
  void pcollect() {
    if (!prof) return;
    sync();
    for (int i = 0; i < pused; ++i) {
      float ms = 0.f;
      HIPC(hipEventElapsedTime(&ms, pev[2 * i], pev[2 * i + 1]));
      pms[pcls[i]] += ms;
      plaunch[pcls[i]] += 1;
    }
    pused = 0;
  }

  template <class T>
  T* dalloc(size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    void* p = nullptr;
    if (alloc.alloc) {
      p = alloc.alloc(alloc.self, bytes, (void*)stream);
      if (!p) fail(SSCF_E_NOMEM, "device allocation of %zu bytes failed", bytes);
    } else {
      const hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) fail(SSCF_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    owned.push_back(p);
    owned_bytes.push_back(bytes);
    return static_cast<T*>(p);
  }

  void dfree(void* p) {
    if (!p) return;
    auto it = std::find(owned.begin(), owned.end(), p);
    if (it == owned.end()) return;
    if (stream) hipStreamSynchronize(stream);
    if (alloc.free) alloc.free(alloc.self, p, (void*)stream);
    else hipFree(p);
    owned_bytes.erase(owned_bytes.begin() + (it - owned.begin()));
    owned.erase(it);
  }

  template <class T>
  T* upload(const T* src, size_t n) {
    T* d = dalloc<T>(n);
    if (n) HIPC(hipMemcpyAsync(d, src, n * sizeof(T), hipMemcpyHostToDevice, stream));
    return d;
  }

  void release() {
    if (stream) hipStreamSynchronize(stream);
    for (void* p : owned) {
      if (alloc.free) alloc.free(alloc.self, p, (void*)stream);
      else hipFree(p);
    }
    owned.clear();
    owned_bytes.clear();
    for (auto& e : ev)
      if (e) { hipEventDestroy(e); e = nullptr; }
    for (auto& e : pev) hipEventDestroy(e);
    pev.clear();
  }

  void sync() { HIPC(hipStreamSynchronize(stream)); }

  Scalars read_scalars() {
    Scalars h{};
    HIPC(hipMemcpyAsync(&h, sd, sizeof(Scalars), hipMemcpyDeviceToHost, stream));
    sync();
    if (h.cap_err) {
      const int64_t t = (int64_t)h.cap_err - 1;
      const int g = (int)(t / v.n_rb), r = (int)(t % v.n_rb);
      double gap = 0.0, R = 0.0;
      if (!cap_R.empty() && g < v.G) {
        const double* a = &cap_gap_g[4 * (size_t)g];
        const double* b = &cap_gap_r[4 * (size_t)r];
        gap = std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2])) -
              a[3] - b[3];
        R = cap_R[g];
      }
      fail(SSCF_E_CAPACITY,
           "a nonzero of C fell on a tile without a slot: group %d, row block %d, %.1f bohr from the group, beyond "
           "its capacity of %.1f bohr (initial reach + slot_margin_bohr)", g, r, gap, R);
    }
    return h;
  }

  // ---------------------------------------------------------------------------------------
  void rebuild_list(int b) { launch_list(v, actC[b], listC[b], cntC[b], stream); }

  // Y = X C on the dilated support of C
  // Y = X C; occ_only: only the occupied columns of every panel are formed
  void product(const double* X, bool dilate, bool occ_only = false) {
    if (dilate) {
      launch_dilate(v, listC[cur], cntC[cur], actY, stream);
      launch_list(v, actY, listY, cntY, stream);
    }
    const unsigned int smask = occ_only ? (1u << (v.OW / 16)) - 1u : 0xffffffffu;
    const int pi = pbegin(KC_SPMM);
    launch_spmm(v, X, C[cur], actC[cur], cmask[cur], listY, cntY, Y, ymask, smask, ctr(KC_SPMM), stream);
    pend(pi);
    if (wc()) count_product(X, C[cur], Y, false, occ_only);
  }

  // orthonormalization loop (section 3.4); returns the number of combination sweeps
  int orthonormalize(int occ_only, int max_sweeps, double* eta_out, int* converged) {
    const double tol = eps / 100.0, cut = 1e-3 * eps;
    int sweeps = 0;
    *converged = 0;
    for (;;) {
      product(S, true, occ_only != 0);
      const int W = v.W;
      const int pi = pbegin(KC_PAIR_O);
      const int nt = (occ_only ? v.OW : W) / 16;
      launch_pair(v, n_pairs, pair_perm, pair_maxc, pg, ph, C[cur], listC[cur], cntC[cur], cmask[cur], Y, actY, ymask, 0, nt, 0, nt, O, W,
                  (size_t)W * W, ctr(KC_PAIR_O), stream);
      pend(pi);
      if (wc()) count_pairs(KC_PAIR_O, n_pairs, pg, ph, C[cur], Y, false, 0, 16 * nt, 0, 16 * nt, 1,
                            overlap_pairs(occ_only != 0));
      HIPC(hipMemsetAsync(&sd->eta_bits, 0, sizeof(unsigned long long), stream));
      HIPC(hipMemsetAsync(&sd->err, 0, sizeof(int), stream));
      launch_ortho_scale(v, v.G, self_pair, O, pnocc, pnvirt, occ_only, sc, sd, stream);
      launch_normalize_d(v, n_pairs, pg, ph, O, Dt, sc, pnocc, pnvirt, occ_only, sd, stream);
      const Scalars h = read_scalars();
      if (h.err & 1) fail(SSCF_E_NOT_SPD, "C^T S C has a non-positive diagonal element");
      double eta;
      std::memcpy(&eta, &h.eta_bits, sizeof(double));
      *eta_out = eta;
      // C's columns are divided by their norms sc: here when the loop ends, else by the packing
      // and the combination as they read C
      const bool last = eta < tol || sweeps >= max_sweeps;
      if (last) {
        launch_scale_c(v, C[cur], listC[cur], cntC[cur], cmask[cur], sc, stream);
        if (eta < tol) *converged = 1;
        break;
      }
      // pair combinations C <- C - 1/2 C D_sel, in place: the combination reads the other
      // groups' tiles from their packed copy, and only the activity flags are double-buffered
      const int nx = 1 - cur;
      HIPC(hipMemsetAsync(upd, 0, (size_t)v.G * W, stream));
      if (wc()) launch_fill_i32(w_nsel, (size_t)v.G * W, 0, stream);
      launch_mark_selected(v, n_pairs, pg, ph, O, sd, pair_sel, upd, rmask, wc() ? w_nsel : nullptr, stream);
      launch_update_support(v, listC[cur], cntC[cur], n_pairs, pg, ph, pair_sel, nullptr, act_tmp, stream);
      launch_list(v, act_tmp, list_tmp, cnt_tmp, stream);
      launch_clear_flags(v, actC[nx], cmask[nx], listC[nx], cntC[nx], stream);
      if (wc()) count_update_begin(occ_only != 0);
      // the combination reads the nonzero columns of C packed into Y (free until the next product)
      const int pu = pbegin(KC_UPDATE);
      launch_pack_cols(v, C[cur], listC[cur], cntC[cur], occ_only ? v.OW : v.W, sc, Y, pcidx, pncol, stream);
      launch_ortho_update(v, C[cur], actC[cur], cmask[cur], Y, pcidx, pncol, gn_ptr, gn, pair_of, pair_sel, O, Dt, rmask, sd, upd,
                          sc, cut, list_tmp, cnt_tmp, C[nx], actC[nx], cmask[nx], ctr(KC_UPDATE), stream);
      pend(pu);
      rebuild_list(nx);
      if (wc()) count_update_end(nx, occ_only != 0);
      cur = nx;
      ++sweeps;
    }
    return sweeps;
  }

  // Mulliken charges from C and Y = S C of the last orthonormalization pass
  void charges(int shift_prev) {
    launch_list_t(v, actC[cur], listT, cntT, stream);
    launch_charges_rows(v, C[cur], listT, cntT, Y, actY, sc, pnocc, rowq, stream);
    HIPC(hipMemsetAsync(&sd->dq_bits, 0, sizeof(unsigned long long), stream));
    launch_atom_charges(v, ao_off, rowq, q, q_prev, dq, sd, shift_prev, stream);
  }

  // Q = gamma dq (kept current in every mode, for the next Fock build), the Coulomb
  // energy and the band energy sum P H0 (or P F with a complete Fock matrix)
  void energy_terms() {
    launch_coulomb(v, scc, dq, part, Q, stream);
    launch_sum_coul(v, scc && !fock_full, dq, Q, sd, stream);
    product(fock_full ? Hfull : H0, false, true);   // support of C unchanged since the last dilation
    launch_coldot(v, C[cur], listC[cur], cntC[cur], cmask[cur], Y, actY, part, dvec, stream);
    launch_sum_band(v, dvec, pnocc, sd, stream);
  }

  // Energy gradient at the current MOs into device buffers (n_val values each; don: 2 per atom,
  // may be NULL), enqueued on the stream.  The charge term of dE/dS only with H0 and SCC.
  void gradient(double* dX, double* dS, double* don) {
    hipStream_t s = stream;
    const size_t fo = (size_t)v.OW * v.OW;
    if (!foo_a) {
      foo_a = dalloc<double>((size_t)n_pairs * fo);
      foo_b = dalloc<double>((size_t)n_pairs * fo);
      wblk = dalloc<double>((size_t)v.nbx * 256);
      pair_all = dalloc<uint8_t>(n_pairs);
      launch_fill_u8(pair_all, n_pairs, 1, s);
    }
    if (!pblk) pblk = dalloc<double>((size_t)v.nbx * 256);
    // the Fock matrix of the current charges, not truncated, and Y = H C_occ
    launch_fock(v, S, H0, fock_full ? Hfull : nullptr, Q, 0.0, H, nullptr, s);
    const bool was = counting;
    counting = false;
    product(H, true, true);
    counting = was;
    // occupied-occupied blocks C_g^T H C_h of every neighbouring pair, in both orientations
    const int no = v.OW / 16;
    launch_pair(v, n_pairs, pair_perm, pair_maxc, pg, ph, C[cur], listC[cur], cntC[cur], cmask[cur], Y, actY, ymask,
                0, no, 0, no, foo_a, v.OW, fo, nullptr, s);
    launch_pair(v, n_pairs, pair_perm, pair_maxc, ph, pg, C[cur], listC[cur], cntC[cur], cmask[cur], Y, actY, ymask,
                0, no, 0, no, foo_b, v.OW, fo, nullptr, s);
    // Z = C_occ F on the row blocks where a neighbouring group is active and that S links to an
    // active row block of the group (W needs no other; Z overwrites Y, in Y's pool)
    launch_update_support(v, listC[cur], cntC[cur], n_pairs, pg, ph, pair_all, actY, act_tmp, s);
    launch_list(v, act_tmp, list_tmp, cnt_tmp, s);
    launch_apply_occ(v, C[cur], actC[cur], cmask[cur], gn_ptr, gn, pair_of, pg, foo_a, foo_b, list_tmp, cnt_tmp, Y, s);
    // P = 2 C_occ C_occ^T and W = 2 C_occ Z^T on the pattern of S, then the layout of S_val
    launch_list_t(v, actC[cur], listT, cntT, s);
    launch_density_blocks(v, C[cur], cmask[cur], listT, cntT, C[cur], actC[cur], cmask[cur], false, pblk, s);
    launch_density_blocks(v, C[cur], cmask[cur], listT, cntT, Y, act_tmp, nullptr, true, wblk, s);
    launch_grad_assemble(v, n_val, val_map, pblk, wblk, Q, scc && !fock_full, dX, dS, s);
    if (don) launch_grad_onsite(v, ao_off, xs_diag, pblk, don, s);
  }

  int64_t active_tiles() {
    std::vector<int> cnt(v.G);
    HIPC(hipMemcpyAsync(cnt.data(), cntC[cur], sizeof(int) * v.G, hipMemcpyDeviceToHost, stream));
    sync();
    int64_t s = 0;
    for (int c : cnt) s += c;
    return s;
  }
};

// =========================================================================================
// set-up
// =========================================================================================

namespace {

// Items of a list sorted by group, laid out so that workgroup L (on XCD L % 8) takes item
// perm[(L % 8) * maxc + L / 8]: every item of group g runs on XCD g % 8, in list order;
// -1 pads the shorter XCD lists.
std::vector<int> xcd_perm(const std::vector<int>& item_group, int* maxc) {
  constexpr int NX = 8;
  std::vector<std::vector<int>> lists(NX);
  for (size_t i = 0; i < item_group.size(); ++i) lists[item_group[i] % NX].push_back((int)i);
  int m = 1;
  for (const auto& l : lists) m = std::max(m, (int)l.size());
  std::vector<int> perm((size_t)NX * m, -1);
  for (int x = 0; x < NX; ++x) std::copy(lists[x].begin(), lists[x].end(), perm.begin() + (size_t)x * m);
  *maxc = m;
  return perm;
}

void validate(const sscf_system_desc* d) {
  if (!d) fail(SSCF_E_INVALID_ARG, "desc is NULL");
  if (d->n_atoms <= 0 || !d->atom_nao || !d->xyz_bohr || !d->hubbard_u || !d->q0 || !d->atom_group)
    fail(SSCF_E_INVALID_ARG, "atom arrays missing or n_atoms <= 0");
  if (d->n_groups <= 0) fail(SSCF_E_INVALID_ARG, "n_groups must be positive");
  if (!d->blk_rowptr || !d->blk_col || !d->blk_off || !d->S_val || !d->H0_val || d->n_val <= 0)
    fail(SSCF_E_INVALID_ARG, "atom-block pattern or values missing");
  if (d->n_mo <= 0 || d->n_occ < 0 || d->n_occ > d->n_mo || !d->mo_group || !d->c0_colptr || !d->c0_row ||
      !d->c0_val)
    fail(SSCF_E_INVALID_ARG, "MO arrays missing or bad n_mo / n_occ");
  if (!(d->eps >= 0.0) || !std::isfinite(d->eps) || !(d->e_conv >= 0.0) || !(d->group_nbr_bohr > 0.0) ||
      !(d->rot_cap_factor >= 0.0) || d->max_sweeps_init < 0 || d->max_sweeps_step < 0)
    fail(SSCF_E_INVALID_ARG, "bad thresholds");
  if (d->precision != SSCF_FP64 && d->precision != SSCF_FP32_MIXED) fail(SSCF_E_INVALID_ARG, "bad precision");
  if (d->flags & ~(uint64_t)(SSCF_FLAG_PROFILE | SSCF_FLAG_COUNT_WORK)) fail(SSCF_E_INVALID_ARG, "unknown bits in flags");
  for (int a = 0; a < d->n_atoms; ++a) {
    if (d->atom_nao[a] < 1 || d->atom_nao[a] > 4) fail(SSCF_E_INVALID_ARG, "atom %d: atom_nao must be 1..4", a);
    if (d->atom_group[a] < 0 || d->atom_group[a] >= d->n_groups) fail(SSCF_E_INVALID_ARG, "atom %d: bad group", a);
    if (!(d->hubbard_u[a] > 0.0) || !std::isfinite(d->hubbard_u[a])) fail(SSCF_E_INVALID_ARG, "atom %d: bad U", a);
    if (!std::isfinite(d->q0[a])) fail(SSCF_E_INVALID_ARG, "atom %d: bad q0", a);
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(d->xyz_bohr[3 * a + k])) fail(SSCF_E_INVALID_ARG, "atom %d: bad position", a);
  }
}

}  // namespace

static void build(sscf_ctx* x, const sscf_system_desc* d) {
  validate(d);
  x->eps = d->eps;
  x->e_conv = d->e_conv;
  x->r_nbr = d->group_nbr_bohr;
  x->rot_cap = d->rot_cap_factor;
  x->max_sweeps_init = d->max_sweeps_init;
  x->max_sweeps_step = d->max_sweeps_step;
  x->scc = d->scc ? 1 : 0;
  x->precision = d->precision;
  x->stream = (hipStream_t)d->hip_stream;
  x->alloc = d->alloc;
  x->n_val = d->n_val;
  x->prof = (d->flags & SSCF_FLAG_PROFILE) != 0;
  x->count = (d->flags & SSCF_FLAG_COUNT_WORK) != 0;
  View& v = x->v;
  const int na = d->n_atoms;
  v.n_atoms = na;
  v.n_mo = d->n_mo;
  v.n_occ = d->n_occ;
  v.G = d->n_groups;
  const int G = v.G;

  // AOs, row blocks
  std::vector<int64_t> ao_off(na + 1, 0);
  for (int a = 0; a < na; ++a) ao_off[a + 1] = ao_off[a] + d->atom_nao[a];
  if (ao_off[na] > (1LL << 30)) fail(SSCF_E_CAPACITY, "too many AOs");
  v.n_ao = (int)ao_off[na];
  v.n_rb = (v.n_ao + RB - 1) / RB;
  std::vector<int> ao_atom(v.n_ao);
  for (int a = 0; a < na; ++a)
    for (int64_t mu = ao_off[a]; mu < ao_off[a + 1]; ++mu) ao_atom[mu] = a;
  x->h_ao_off = ao_off;

  // atom-block pattern: checks, symmetry, and the row-block pattern
  const int64_t* rp = d->blk_rowptr;
  if (rp[0] != 0) fail(SSCF_E_INVALID_ARG, "blk_rowptr[0] must be 0");
  for (int a = 0; a < na; ++a) {
    if (rp[a + 1] < rp[a]) fail(SSCF_E_INVALID_ARG, "blk_rowptr must not decrease");
    bool self = false;
    for (int64_t k = rp[a]; k < rp[a + 1]; ++k) {
      const int b = d->blk_col[k];
      if (b < 0 || b >= na || (k > rp[a] && d->blk_col[k - 1] >= b))
        fail(SSCF_E_INVALID_ARG, "row %d of the atom-block pattern: columns must be in range and increasing", a);
      if (b == a) self = true;
      const int64_t end = d->blk_off[k] + (int64_t)d->atom_nao[a] * d->atom_nao[b];
      if (d->blk_off[k] < 0 || end > d->n_val) fail(SSCF_E_INVALID_ARG, "block (%d, %d) outside the values", a, b);
      for (int64_t t = d->blk_off[k]; t < end; ++t)
        if (!std::isfinite(d->S_val[t]) || !std::isfinite(d->H0_val[t]))
          fail(SSCF_E_INVALID_ARG, "non-finite S or H0 in block (%d, %d)", a, b);
    }
    if (!self) fail(SSCF_E_INVALID_ARG, "atom %d has no self block", a);
  }
  auto find_blk = [&](int a, int b) -> int64_t {
    const int32_t* lo = d->blk_col + rp[a];
    const int32_t* hi = d->blk_col + rp[a + 1];
    const int32_t* it = std::lower_bound(lo, hi, b);
    return (it != hi && *it == b) ? (int64_t)(it - d->blk_col) : -1;
  };
  for (int a = 0; a < na; ++a)
    for (int64_t k = rp[a]; k < rp[a + 1]; ++k) {
      const int b = d->blk_col[k];
      const int64_t kt = find_blk(b, a);
      if (kt < 0) fail(SSCF_E_INVALID_ARG, "atom-block pattern is not symmetric at (%d, %d)", a, b);
      const int nA = d->atom_nao[a], nB = d->atom_nao[b];
      for (int i = 0; i < nA; ++i)
        for (int j = 0; j < nB; ++j) {
          const int64_t s1 = d->blk_off[k] + (int64_t)i * nB + j, s2 = d->blk_off[kt] + (int64_t)j * nA + i;
          if (d->S_val[s1] != d->S_val[s2] || d->H0_val[s1] != d->H0_val[s2])
            fail(SSCF_E_INVALID_ARG, "S and H0 must be symmetric (atoms %d, %d)", a, b);
        }
    }
  // row-block pattern (r, c) covered by any atom block
  std::vector<std::vector<int>> rbcols(v.n_rb);
  for (int a = 0; a < na; ++a)
    for (int64_t k = rp[a]; k < rp[a + 1]; ++k) {
      const int b = d->blk_col[k];
      for (int64_t r = ao_off[a] / RB; r <= (ao_off[a + 1] - 1) / RB; ++r)
        for (int64_t c = ao_off[b] / RB; c <= (ao_off[b + 1] - 1) / RB; ++c) rbcols[r].push_back((int)c);
    }
  std::vector<int> xs_ptr(v.n_rb + 1, 0), xs_col, xs_row;
  for (int r = 0; r < v.n_rb; ++r) {
    auto& cs = rbcols[r];
    std::sort(cs.begin(), cs.end());
    cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
    for (int c : cs) { xs_col.push_back(c); xs_row.push_back(r); }
    xs_ptr[r + 1] = (int)xs_col.size();
  }
  v.nbx = (int)xs_col.size();
  auto xs_find = [&](int r, int c) -> int64_t {
    auto lo = xs_col.begin() + xs_ptr[r], hi = xs_col.begin() + xs_ptr[r + 1];
    auto it = std::lower_bound(lo, hi, c);
    return (int64_t)(it - xs_col.begin());
  };
  std::vector<int64_t> val_map(d->n_val, -1);
  for (int a = 0; a < na; ++a)
    for (int64_t k = rp[a]; k < rp[a + 1]; ++k) {
      const int b = d->blk_col[k];
      const int nA = d->atom_nao[a], nB = d->atom_nao[b];
      for (int i = 0; i < nA; ++i)
        for (int j = 0; j < nB; ++j) {
          const int64_t mu = ao_off[a] + i, nu = ao_off[b] + j;
          const int64_t bi = xs_find((int)(mu / RB), (int)(nu / RB));
          val_map[d->blk_off[k] + (int64_t)i * nB + j] = bi * 256 + (mu % RB) * 16 + (nu % RB);
        }
    }
  for (int64_t t = 0; t < d->n_val; ++t)
    if (val_map[t] < 0) fail(SSCF_E_INVALID_ARG, "value %lld of S_val is not covered by any block", (long long)t);

  // MO panels (section 3.2: MOs keep their group)
  std::vector<int> nocc(G, 0), nvirt(G, 0), mo_col(v.n_mo);
  for (int j = 0; j < v.n_mo; ++j) {
    const int g = d->mo_group[j];
    if (g < 0 || g >= G) fail(SSCF_E_INVALID_ARG, "MO %d: bad group", j);
    mo_col[j] = (j < v.n_occ) ? nocc[g]++ : nvirt[g]++;
  }
  int mo_ = 0, mv_ = 0;
  for (int g = 0; g < G; ++g) { mo_ = std::max(mo_, nocc[g]); mv_ = std::max(mv_, nvirt[g]); }
  v.OW = std::max(16, round16(mo_));
  v.VW = std::max(16, round16(mv_));
  v.W = v.OW + v.VW;
  if (v.W > MAX_W) fail(SSCF_E_CAPACITY, "MO group too large: %d + %d MOs (panel limit %d)", mo_, mv_, MAX_W);
  std::vector<int> mo_panel(v.n_mo);
  x->h_mo_of.assign((size_t)G * v.W, -1);
  for (int j = 0; j < v.n_mo; ++j) {
    mo_panel[j] = d->mo_group[j];
    if (j >= v.n_occ) mo_col[j] += v.OW;
    x->h_mo_of[(size_t)mo_panel[j] * v.W + mo_col[j]] = j;
  }
  x->h_pnocc = nocc;
  x->h_pnvirt = nvirt;

  // C0 checks
  const int64_t* cp = d->c0_colptr;
  if (cp[0] != 0) fail(SSCF_E_INVALID_ARG, "c0_colptr[0] must be 0");
  for (int j = 0; j < v.n_mo; ++j) {
    if (cp[j + 1] < cp[j]) fail(SSCF_E_INVALID_ARG, "c0_colptr must not decrease");
    for (int64_t t = cp[j]; t < cp[j + 1]; ++t) {
      if (d->c0_row[t] < 0 || d->c0_row[t] >= v.n_ao || (t > cp[j] && d->c0_row[t] <= d->c0_row[t - 1]))
        fail(SSCF_E_INVALID_ARG, "C0 column %d: rows must be increasing and in range", j);
      if (!std::isfinite(d->c0_val[t])) fail(SSCF_E_INVALID_ARG, "C0 column %d: non-finite value", j);
    }
  }
  const int64_t nnz0 = cp[v.n_mo];
  if (nnz0 > (1LL << 31) - 1) fail(SSCF_E_CAPACITY, "C0 too large");

  // group neighbour map: some atom pair closer than r_nbr (section 3.2), on the GPU
  std::vector<uint8_t> gnbr((size_t)G * G, 0);
  {
    std::vector<int> ga_ptr(G + 1, 0), ga(na), fillp(G, 0);
    for (int a = 0; a < na; ++a) ga_ptr[d->atom_group[a] + 1]++;
    for (int g = 0; g < G; ++g) ga_ptr[g + 1] += ga_ptr[g];
    for (int a = 0; a < na; ++a) ga[ga_ptr[d->atom_group[a]] + fillp[d->atom_group[a]]++] = a;
    double* dxyz = x->upload(d->xyz_bohr, (size_t)3 * na);
    int* dag = x->upload(d->atom_group, (size_t)na);
    int* dgp = x->upload(ga_ptr.data(), ga_ptr.size());
    int* dga = x->upload(ga.data(), ga.size());
    uint8_t* dn = x->dalloc<uint8_t>((size_t)G * G);
    launch_fill_u8(dn, (size_t)G * G, 0, x->stream);
    launch_group_nbr(na, G, dxyz, dag, dgp, dga, x->r_nbr, dn, x->stream);
    HIPC(hipMemcpyAsync(gnbr.data(), dn, (size_t)G * G, hipMemcpyDeviceToHost, x->stream));
    x->sync();
    x->dfree(dxyz); x->dfree(dag); x->dfree(dgp); x->dfree(dga); x->dfree(dn);
    // the relation is symmetric by construction; keep it exactly so
    for (int g = 0; g < G; ++g)
      for (int h2 = g + 1; h2 < G; ++h2) {
        const uint8_t e = gnbr[(size_t)g * G + h2] | gnbr[(size_t)h2 * G + g];
        gnbr[(size_t)g * G + h2] = gnbr[(size_t)h2 * G + g] = e;
      }
  }
  std::vector<int> gn_ptr(G + 1, 0), gn;
  for (int g = 0; g < G; ++g) {
    for (int h = 0; h < G; ++h)
      if (gnbr[(size_t)g * G + h]) gn.push_back(h);
    gn_ptr[g + 1] = (int)gn.size();
  }
  // unordered pairs g <= h
  std::vector<int> pg, ph, pair_of((size_t)G * G, -1), self_pair(G, -1);
  for (int g = 0; g < G; ++g)
    for (int h = g; h < G; ++h)
      if (gnbr[(size_t)g * G + h]) {
        pair_of[(size_t)g * G + h] = pair_of[(size_t)h * G + g] = (int)pg.size();
        if (g == h) self_pair[g] = (int)pg.size();
        pg.push_back(g);
        ph.push_back(h);
      }
  // the rotation pass keeps two 64-bit column masks per group in LDS (64 KB per workgroup)
  if (256 * 16 + 16 * (size_t)G + 4 * 128 + 16 > 65536) fail(SSCF_E_CAPACITY, "%d MO groups: at most 3800", G);
  x->n_pairs = (int)pg.size();
  x->h_pg = pg;
  x->h_ph = ph;
  // Jacobi blocks (g occupied, h virtual), greedy rounds in (g, h) order (section 3.5)
  {
    int maxdeg = 0;
    for (int g = 0; g < G; ++g) maxdeg = std::max(maxdeg, gn_ptr[g + 1] - gn_ptr[g]);
    const int RMAX = 2 * maxdeg + 2;
    std::vector<uint8_t> used_o((size_t)G * RMAX, 0), used_v((size_t)G * RMAX, 0);
    for (int g = 0; g < G; ++g) {
      if (nocc[g] == 0) continue;
      for (int k = gn_ptr[g]; k < gn_ptr[g + 1]; ++k) {
        const int h = gn[k];
        if (nvirt[h] == 0) continue;
        int r = 0;
        while (used_o[(size_t)g * RMAX + r] || used_v[(size_t)h * RMAX + r]) ++r;
        used_o[(size_t)g * RMAX + r] = used_v[(size_t)h * RMAX + r] = 1;
        x->h_jb_g.push_back(g);
        x->h_jb_h.push_back(h);
        x->h_jb_round.push_back(r);
        x->n_rounds = std::max(x->n_rounds, r + 1);
      }
    }
    x->n_blocks = (int)x->h_jb_g.size();
    x->h_round_ptr.assign(x->n_rounds + 1, 0);
    for (int r : x->h_jb_round) x->h_round_ptr[r + 1]++;
    for (int r = 0; r < x->n_rounds; ++r) x->h_round_ptr[r + 1] += x->h_round_ptr[r];
  }
  std::vector<int> round_list(x->n_blocks), jb_nocc(x->n_blocks), jb_nvirt(x->n_blocks);
  {
    std::vector<int> fillp(x->h_round_ptr.begin(), x->h_round_ptr.end() - 1);
    for (int b = 0; b < x->n_blocks; ++b) {
      round_list[fillp[x->h_jb_round[b]]++] = b;
      jb_nocc[b] = nocc[x->h_jb_g[b]];
      jb_nvirt[b] = nvirt[x->h_jb_h[b]];
    }
  }

  // ---- device memory -------------------------------------------------------------------
  for (auto& e : x->ev) HIPC(hipEventCreate(&e));
  hipStream_t s = x->stream;
  x->xyz = x->upload(d->xyz_bohr, (size_t)3 * na);
  x->U = x->upload(d->hubbard_u, na);
  x->q0 = x->upload(d->q0, na);
  x->ao_atom = x->upload(ao_atom.data(), ao_atom.size());
  x->ao_off = x->upload(ao_off.data(), ao_off.size());
  x->xs_ptr = x->upload(xs_ptr.data(), xs_ptr.size());
  x->xs_col = x->upload(xs_col.data(), xs_col.size());
  x->xs_row = x->upload(xs_row.data(), xs_row.size());
  {
    std::vector<int> diag(v.n_rb);
    for (int r = 0; r < v.n_rb; ++r) diag[r] = (int)xs_find(r, r);
    x->xs_diag = x->upload(diag.data(), diag.size());
  }
  x->val_map = x->upload(val_map.data(), val_map.size());
  v.xyz = x->xyz;
  v.U = x->U;
  v.q0 = x->q0;
  v.ao_atom = x->ao_atom;
  v.xs_ptr = x->xs_ptr;
  v.xs_col = x->xs_col;
  v.xs_row = x->xs_row;
  const size_t nxe = (size_t)v.nbx * 256;
  x->S = x->dalloc<double>(nxe);
  x->H0 = x->dalloc<double>(nxe);
  x->H = x->dalloc<double>(nxe);
  HIPC(hipMemsetAsync(x->S, 0, nxe * sizeof(double), s));
  HIPC(hipMemsetAsync(x->H0, 0, nxe * sizeof(double), s));
  {
    double* tmp = x->upload(d->S_val, d->n_val);
    launch_scatter(x->val_map, d->n_val, tmp, x->S, s);
    x->dfree(tmp);
    tmp = x->upload(d->H0_val, d->n_val);
    launch_scatter(x->val_map, d->n_val, tmp, x->H0, s);
    x->dfree(tmp);
  }
  x->h_blk_rowptr.assign(rp, rp + na + 1);
  x->h_blk_col.assign(d->blk_col, d->blk_col + rp[na]);
  x->h_blk_off.assign(d->blk_off, d->blk_off + rp[na]);
  x->h_atom_nao.assign(d->atom_nao, d->atom_nao + na);
  const size_t ntiles = (size_t)G * v.n_rb;
  const size_t tile_elems = (size_t)RB * v.W;
  // Tile capacity.  Without a margin every tile (g, r) has a slot (dense capacity,
  // 8 G n_rb 16 W bytes per copy of C).  With one, group g gets the row blocks within
  // R_g = reach_g + margin of it, reach_g the farthest row block that g's initial MOs touch
  // (section 3.2: the MOs of a group stay near it).  Distances are taken between bounding
  // spheres (of the group's atoms, of the block's atoms), a superset of the atom-to-atom test;
  // memory then grows with the number of atoms instead of its square.
  {
    std::vector<int> slot(ntiles, -1);
    int64_t ns = 0;
    if (!(d->slot_margin_bohr > 0.0)) {
      for (size_t t = 0; t < ntiles; ++t) slot[t] = (int)t;
      ns = (int64_t)ntiles;
    } else {
      auto sphere = [&](const std::vector<int>& atoms, double* c) {
        c[0] = c[1] = c[2] = 0.0;
        for (int a : atoms)
          for (int k = 0; k < 3; ++k) c[k] += d->xyz_bohr[3 * a + k];
        for (int k = 0; k < 3; ++k) c[k] /= (double)atoms.size();
        double r2 = 0.0;
        for (int a : atoms) {
          double q = 0.0;
          for (int k = 0; k < 3; ++k) q += (d->xyz_bohr[3 * a + k] - c[k]) * (d->xyz_bohr[3 * a + k] - c[k]);
          r2 = std::max(r2, q);
        }
        c[3] = std::sqrt(r2);
      };
      std::vector<std::vector<int>> gat(G), rat(v.n_rb);
      for (int a = 0; a < na; ++a) {
        gat[d->atom_group[a]].push_back(a);
        for (int64_t r = ao_off[a] / RB; r <= (ao_off[a + 1] - 1) / RB; ++r) rat[r].push_back(a);
      }
      std::vector<double> gs((size_t)G * 4, 0.0), rs((size_t)v.n_rb * 4, 0.0);
      for (int g = 0; g < G; ++g)
        if (!gat[g].empty()) sphere(gat[g], &gs[4 * (size_t)g]);
      for (int r = 0; r < v.n_rb; ++r) sphere(rat[r], &rs[4 * (size_t)r]);
      auto gap = [&](int g, int r) {
        const double* a = &gs[4 * (size_t)g];
        const double* b = &rs[4 * (size_t)r];
        const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
        return std::sqrt(dx * dx + dy * dy + dz * dz) - a[3] - b[3];
      };
      std::vector<double> reach(G, 0.0);
      for (int j = 0; j < v.n_mo; ++j) {
        const int g = d->mo_group[j];
        int last = -1;
        for (int64_t t = cp[j]; t < cp[j + 1]; ++t) {
          const int r = d->c0_row[t] / RB;
          if (r == last || d->c0_val[t] == 0.0) continue;
          last = r;
          reach[g] = std::max(reach[g], gap(g, r));
        }
      }
      x->cap_gap_g = gs;
      x->cap_gap_r = rs;
      x->cap_R.assign(G, 0.0);
      for (int g = 0; g < G; ++g) {
        if (gat[g].empty()) continue;
        const double R = reach[g] + d->slot_margin_bohr;
        x->cap_R[g] = R;
        for (int r = 0; r < v.n_rb; ++r) {
          if (gap(g, r) < R) {
            if (ns >= INT32_MAX) fail(SSCF_E_CAPACITY, "more than 2^31 tile slots");
            slot[(size_t)g * v.n_rb + r] = (int)ns++;
          }
        }
      }
    }
    x->n_slots = (size_t)std::max<int64_t>(ns, 1);
    x->slot = x->upload(slot.data(), slot.size());
    v.slot = x->slot;
    // the pools of Y = X C: every row block that X's pattern links to a row block where C has
    // a slot (Y never has a nonzero elsewhere)
    std::vector<int> slotY(ntiles, -1);
    int64_t nsy = 0;
    if (!(d->slot_margin_bohr > 0.0)) {
      slotY = slot;
      nsy = ns;
    } else {
      for (int g = 0; g < G; ++g) {
        const int* sg = &slot[(size_t)g * v.n_rb];
        for (int r = 0; r < v.n_rb; ++r) {
          bool need = sg[r] >= 0;
          for (int k = xs_ptr[r]; k < xs_ptr[r + 1] && !need; ++k) need = sg[xs_col[k]] >= 0;
          if (need) {
            if (nsy >= INT32_MAX) fail(SSCF_E_CAPACITY, "more than 2^31 tile slots");
            slotY[(size_t)g * v.n_rb + r] = (int)nsy++;
          }
        }
      }
    }
    x->n_slots_y = (size_t)std::max<int64_t>(nsy, 1);
    x->slotY = x->upload(slotY.data(), slotY.size());
    v.slotY = x->slotY;
    v.max_c = v.max_y = 1;
    for (int g = 0; g < G; ++g) {
      int nc = 0, ny = 0;
      for (int r = 0; r < v.n_rb; ++r) {
        nc += slot[(size_t)g * v.n_rb + r] >= 0;
        ny += slotY[(size_t)g * v.n_rb + r] >= 0;
      }
      v.max_c = std::max(v.max_c, nc);
      v.max_y = std::max(v.max_y, ny);
    }
  }
  const size_t nslot = x->n_slots, nslot_y = x->n_slots_y;
  // one pool of C values (C[0] and C[1] are the same memory: see orthonormalize), two sets of
  // activity flags and lists
  x->C[0] = x->C[1] = x->dalloc<double>(nslot * tile_elems);
  HIPC(hipMemsetAsync(x->C[0], 0, nslot * tile_elems * sizeof(double), s));
  for (int b = 0; b < 2; ++b) {
    x->actC[b] = x->dalloc<uint8_t>(ntiles);
    HIPC(hipMemsetAsync(x->actC[b], 0, ntiles, s));
    x->listC[b] = x->dalloc<int>(ntiles);
    x->cmask[b] = x->dalloc<unsigned int>(ntiles);
    HIPC(hipMemsetAsync(x->cmask[b], 0, ntiles * sizeof(unsigned int), s));
    x->cntC[b] = x->dalloc<int>(G);
    HIPC(hipMemsetAsync(x->cntC[b], 0, sizeof(int) * G, s));
  }
  x->Y = x->dalloc<double>(nslot_y * tile_elems);
  x->actY = x->dalloc<uint8_t>(ntiles);
  x->ymask = x->dalloc<unsigned int>(ntiles);
  x->listY = x->dalloc<int>(ntiles);
  x->cntY = x->dalloc<int>(G);
  x->act_tmp = x->dalloc<uint8_t>(ntiles);
  x->list_tmp = x->dalloc<int>(ntiles);
  x->cnt_tmp = x->dalloc<int>(G);
  x->listT = x->dalloc<int>(ntiles);
  x->cntT = x->dalloc<int>(v.n_rb);
  x->pnocc = x->upload(nocc.data(), G);
  x->pnvirt = x->upload(nvirt.data(), G);
  x->mo_of = x->upload(x->h_mo_of.data(), x->h_mo_of.size());
  x->gn_ptr = x->upload(gn_ptr.data(), gn_ptr.size());
  x->gn = x->upload(gn.data(), gn.size());
  x->pair_of = x->upload(pair_of.data(), pair_of.size());
  x->pg = x->upload(pg.data(), pg.size());
  {
    std::vector<int> perm = xcd_perm(pg, &x->pair_maxc);
    x->pair_perm = x->upload(perm.data(), perm.size());
  }
  x->ph = x->upload(ph.data(), ph.size());
  x->self_pair = x->upload(self_pair.data(), self_pair.size());
  x->O = x->dalloc<double>((size_t)x->n_pairs * v.W * v.W);
  x->Dt = x->dalloc<double>((size_t)x->n_pairs * v.W * v.W);
  x->sc = x->dalloc<double>((size_t)G * v.W);
  x->upd = x->dalloc<uint8_t>((size_t)G * v.W);
  x->pair_sel = x->dalloc<uint8_t>(x->n_pairs);
  x->rmask = x->dalloc<uint8_t>((size_t)x->n_pairs * 2 * v.W);
  x->pcidx = x->dalloc<uint8_t>(nslot_y * v.W);
  x->pncol = x->dalloc<uint8_t>(ntiles);
  {
    double* z = x->dalloc<double>(ZERO_DOUBLES);
    launch_fill(z, ZERO_DOUBLES, 0.0, s);
    v.zeros = z;
  }
  x->part = x->dalloc<double>(std::max((size_t)CD_SPLIT * x->v.G * x->v.W, (size_t)CL_SPLIT * x->v.n_atoms));
  x->jb_g = x->upload(x->h_jb_g.data(), x->n_blocks);
  {
    std::vector<int> perm = xcd_perm(x->h_jb_g, &x->jb_maxc);
    x->jb_perm = x->upload(perm.data(), perm.size());
  }
  x->jb_h = x->upload(x->h_jb_h.data(), x->n_blocks);
  x->jb_nocc = x->upload(jb_nocc.data(), x->n_blocks);
  x->jb_nvirt = x->upload(jb_nvirt.data(), x->n_blocks);
  x->round_list = x->upload(round_list.data(), x->n_blocks);
  const size_t per = (size_t)v.OW * v.VW;
  x->F = x->dalloc<double>((size_t)x->n_blocks * per);
  x->Fdiag = x->dalloc<double>((size_t)G * v.W);
  x->dvec = x->dalloc<double>((size_t)G * v.W);
  x->rot_cnt = x->dalloc<int>(x->n_blocks);
  HIPC(hipMemsetAsync(x->rot_cnt, 0, sizeof(int) * x->n_blocks, s));
  x->rot_slot = x->dalloc<int2>((size_t)x->n_blocks * per);
  if (x->precision == SSCF_FP32_MIXED) {
    x->H32 = x->dalloc<float>(nxe);
    // C32 and Y32 live only inside the C^T H C pass, when Y holds nothing that is read later
    // (every later reader of Y recomputes it first): they share Y's memory, nslot + nslot_y FP32
    // tiles within its nslot_y FP64 tiles (nslot <= nslot_y)
    x->C32 = reinterpret_cast<float*>(x->Y);
    x->Y32 = reinterpret_cast<float*>(x->Y) + nslot_y * tile_elems;
    x->R32 = x->dalloc<float>((size_t)x->n_blocks * v.W * v.W);
  } else {
    x->Rrot = x->dalloc<double>((size_t)x->n_blocks * v.W * v.W);
  }
  x->round_ptr = x->upload(x->h_round_ptr.data(), x->h_round_ptr.size());
  x->rcnt = x->dalloc<int>(x->n_rounds + 1);
  x->roff = x->dalloc<int>(x->n_rounds + 1);
  x->rmeta = x->dalloc<int4>(x->n_blocks);
  x->rot_cs = x->dalloc<double2>((size_t)x->n_blocks * per);
  x->tcnt = x->dalloc<int>(x->n_blocks);
  x->tcol = x->dalloc<int>((size_t)x->n_blocks * v.W);
  x->tmask = x->dalloc<ulonglong2>(x->n_blocks);
  x->colm = x->dalloc<ulonglong2>(ntiles);
  x->hist = x->dalloc<unsigned int>(256);
  HIPC(hipMemsetAsync(x->hist, 0, 256 * sizeof(unsigned int), s));
  x->ties = x->dalloc<long long>(MAX_TIES);
  x->q = x->dalloc<double>(na);
  x->q_prev = x->dalloc<double>(na);
  x->dq = x->dalloc<double>(na);
  x->Q = x->dalloc<double>(na);
  HIPC(hipMemsetAsync(x->q, 0, sizeof(double) * na, s));
  x->rowq = x->dalloc<double>(v.n_ao);
  x->sd = x->dalloc<Scalars>(1);
  HIPC(hipMemsetAsync(x->sd, 0, sizeof(Scalars), s));
  v.cap_err = &x->sd->cap_err;
  x->pctr = x->dalloc<unsigned long long>(SSCF_N_KERNEL_CLASSES);
  HIPC(hipMemsetAsync(x->pctr, 0, sizeof(unsigned long long) * SSCF_N_KERNEL_CLASSES, s));
  if (x->count) {
    x->wdev = x->dalloc<unsigned long long>(8);
    x->w_xrow = x->dalloc<int>((size_t)v.n_rb * RB);
    x->w_colnnz = x->dalloc<int>((size_t)G * v.W);
    x->w_nsel = x->dalloc<int>((size_t)G * v.W);
    x->w_mC = x->dalloc<ulonglong2>(nslot * RB);
    x->w_mY = x->dalloc<ulonglong2>(nslot_y * RB);
  }

  // C0 into the tiles
  {
    std::vector<int64_t> col_of(nnz0);
    for (int j = 0; j < v.n_mo; ++j)
      for (int64_t t = cp[j]; t < cp[j + 1]; ++t) col_of[t] = j;
    int64_t* dcol = x->upload(col_of.data(), nnz0);
    int* drow = x->upload(d->c0_row, nnz0);
    double* dval = x->upload(d->c0_val, nnz0);
    int* dpanel = x->upload(mo_panel.data(), v.n_mo);
    int* dcolm = x->upload(mo_col.data(), v.n_mo);
    launch_scatter_c0(v, (int)nnz0, dcol, drow, dval, dpanel, dcolm, x->C[0], x->actC[0], x->cmask[0], v.cap_err, s);
    x->cur = 0;
    x->rebuild_list(0);
    x->dfree(dcol); x->dfree(drow); x->dfree(dval); x->dfree(dpanel); x->dfree(dcolm);
  }
  x->sync();

  // initial orthonormalization (section 3.4), charges and energy
  x->counting = true;
  HIPC(hipEventRecord(x->ev[0], s));
  double eta = 0.0;
  int conv = 0;
  const int sweeps = x->orthonormalize(0, x->max_sweeps_init, &eta, &conv);
  if (!conv) fail(SSCF_E_ORTHO, "initial orthonormalization did not reach eps/100 in %d sweeps (eta %.3e)", sweeps, eta);
  x->charges(0);
  HIPC(hipMemcpyAsync(x->q_prev, x->q, sizeof(double) * na, hipMemcpyDeviceToDevice, s));
  x->energy_terms();
  HIPC(hipEventRecord(x->ev[1], s));
  const Scalars h = x->read_scalars();
  x->E = h.e_band + h.e_coul;
  sscf_step_info& ii = x->init_info;
  std::memset(&ii, 0, sizeof(ii));
  ii.energy = x->E;
  ii.e_band = h.e_band;
  ii.e_coul = h.e_coul;
  ii.ortho_eta = eta;
  ii.n_ortho_sweeps = sweeps;
  ii.ortho_converged = conv;
  ii.nnz_tiles = x->active_tiles();
  ii.nnz_c = x->count ? x->count_nnz_c() : -1;
  x->counting = false;
  float ms = 0.f;
  HIPC(hipEventElapsedTime(&ms, x->ev[0], x->ev[1]));
  ii.ms_ortho = ms;
  ii.ms_total = ms;
  x->pcollect();
}

// one SCF step
static void step(sscf_ctx* x, sscf_step_info* out) {
  View& v = x->v;
  hipStream_t s = x->stream;
  sscf_step_info info;
  std::memset(&info, 0, sizeof(info));
  x->counting = true;
  const double E_prev = x->E;
  HIPC(hipMemsetAsync(x->sd, 0, offsetof(Scalars, e_band), s));
  HIPC(hipEventRecord(x->ev[0], s));
  // step IV: Fock matrix with the charges of the previous step (Q = gamma dq)
  int pi = x->pbegin(KC_FOCK);
  launch_fock(v, x->S, x->H0, x->fock_full ? x->Hfull : nullptr, x->Q, x->eps, x->H, x->H32, s);
  x->pend(pi);
  HIPC(hipEventRecord(x->ev[1], s));
  // C^T H C: occupied-virtual blocks and the diagonal (FP32 in the precision form)
  if (x->precision == SSCF_FP32_MIXED) {
    launch_dilate(v, x->listC[x->cur], x->cntC[x->cur], x->actY, s);
    launch_list(v, x->actY, x->listY, x->cntY, s);
    pi = x->pbegin(KC_SPMM);
    launch_round_c32(v, x->C[x->cur], x->listC[x->cur], x->cntC[x->cur], x->cmask[x->cur], x->C32, s);
    launch_spmm32(v, x->H32, x->C32, x->actC[x->cur], x->cmask[x->cur], x->listY, x->cntY, x->Y32, x->ymask,
                  x->ctr(KC_SPMM), s);
    x->pend(pi);
    if (x->wc()) x->count_product(x->H32, x->C32, x->Y32, true, false);
    pi = x->pbegin(KC_PAIR_F);
    launch_pair32(v, x->n_blocks, x->jb_perm, x->jb_maxc, x->jb_g, x->jb_h, x->C32, x->listC[x->cur], x->cntC[x->cur],
                  x->cmask[x->cur], x->Y32, x->actY, x->ymask, 0, v.OW / 16, v.OW, v.VW / 16, x->F, v.VW,
                  (size_t)v.OW * v.VW, x->ctr(KC_PAIR_F), s);
    x->pend(pi);
    if (x->wc())
      x->count_pairs(KC_PAIR_F, x->n_blocks, x->jb_g, x->jb_h, x->C32, x->Y32, true, 0, v.OW, v.OW, v.W, 0,
                     x->fock_pairs());
    launch_coldot32(v, x->C32, x->listC[x->cur], x->cntC[x->cur], x->cmask[x->cur], x->Y32, x->actY, x->Fdiag, s);
  } else {
    x->product(x->H, true);
    pi = x->pbegin(KC_PAIR_F);
    launch_pair(v, x->n_blocks, x->jb_perm, x->jb_maxc, x->jb_g, x->jb_h, x->C[x->cur], x->listC[x->cur], x->cntC[x->cur],
                x->cmask[x->cur], x->Y, x->actY, x->ymask, 0, v.OW / 16, v.OW, v.VW / 16, x->F, v.VW,
                (size_t)v.OW * v.VW, x->ctr(KC_PAIR_F), s);
    x->pend(pi);
    if (x->wc())
      x->count_pairs(KC_PAIR_F, x->n_blocks, x->jb_g, x->jb_h, x->C[x->cur], x->Y, false, 0, v.OW, v.OW, v.W, 0,
                     x->fock_pairs());
    launch_coldot(v, x->C[x->cur], x->listC[x->cur], x->cntC[x->cur], x->cmask[x->cur], x->Y, x->actY, x->part,
                  x->Fdiag, s);
  }
  HIPC(hipEventRecord(x->ev[2], s));
  // step V: selection of the rotations
  pi = x->pbegin(KC_SELECT);
  launch_count_candidates(x->n_blocks, v.OW, v.VW, x->jb_nocc, x->jb_nvirt, x->F, x->eps, x->sd, s);
  x->pend(pi);
  int n_cand = 0;
  HIPC(hipMemcpyAsync(&n_cand, &x->sd->n_cand, sizeof(int), hipMemcpyDeviceToHost, s));
  x->sync();
  const long long K = (long long)std::floor(x->rot_cap * v.n_occ);
  pi = x->pbegin(KC_SELECT);
  if (n_cand <= K) {
    launch_sel_init(x->sd, K, 1, s);
  } else {
    launch_sel_init(x->sd, K, 0, s);
    for (int shift = 56; shift >= 0; shift -= 8)
      launch_radix_pass(x->n_blocks, v.OW, v.VW, x->jb_nocc, x->jb_nvirt, x->F, x->eps, shift, x->sd, x->hist, s);
    launch_sel_finish(x->sd, s);
    launch_tie_cut(x->n_blocks, v.OW, v.VW, x->jb_g, x->jb_h, x->jb_nocc, x->jb_nvirt, x->F, x->mo_of, v.W, v.n_mo,
                   x->eps, x->sd, x->ties, s);
  }
  launch_block_select(v, x->n_blocks, x->jb_g, x->jb_h, x->jb_nocc, x->jb_nvirt, x->F, x->Fdiag, x->mo_of, x->eps,
                      x->sd, x->rot_cnt, x->rot_slot, x->rot_cs, x->tcnt, x->tcol, x->tmask,
                      x->precision == SSCF_FP32_MIXED, s);
  x->pend(pi);
  HIPC(hipEventRecord(x->ev[3], s));
  // rotations: composed per block, applied in one pass over the row blocks
  pi = x->pbegin(KC_GIVENS);
  launch_compose_rot(v, x->n_blocks, x->rot_cnt, x->rot_slot, x->rot_cs, x->tcnt, x->Rrot, x->R32, s);
  launch_round_meta(x->n_rounds, x->round_ptr, x->round_list, x->rot_cnt, x->jb_g, x->jb_h, x->tcnt, x->rcnt,
                    x->roff, x->rmeta, s);
  if (x->wc()) x->wzero();
  // the nonzero columns of every active tile, kept exact by the pass (which also leaves exact
  // tile flags: the cut |C| < eps can empty a tile or a slice)
  launch_tile_flags(v, x->C[x->cur], x->listC[x->cur], x->cntC[x->cur], x->actC[x->cur], x->cmask[x->cur], x->colm, s);
  launch_givens_rb(v, x->n_rounds, x->roff, x->rmeta, x->tmask, x->tcol, x->Rrot, x->R32, x->eps, x->C[x->cur],
                   x->actC[x->cur], x->cmask[x->cur], x->colm, x->rot_cnt, x->wc() ? x->wdev : nullptr, s);
  x->pend(pi);
  x->rebuild_list(x->cur);
  if (x->wc()) {
    const auto w = x->wread();
    x->wfl[KC_GIVENS] += (double)w[0];
    x->wby[KC_GIVENS] += (double)w[1];
  }
  HIPC(hipEventRecord(x->ev[4], s));
  // step III: re-orthonormalization
  double eta = 0.0;
  int conv = 0;
  if (x->step_ortho) {
    info.n_ortho_sweeps = x->orthonormalize(0, x->max_sweeps_step, &eta, &conv);
  } else {
    // no step III: the charges take S C of the rotated MOs as they are
    x->product(x->S, true, true);
    launch_fill(x->sc, (size_t)v.G * v.W, 1.0, s);
  }
  info.ortho_eta = eta;
  info.ortho_converged = conv;
  HIPC(hipEventRecord(x->ev[5], s));
  // charges, Coulomb term, energy
  x->charges(1);
  x->energy_terms();
  HIPC(hipEventRecord(x->ev[6], s));
  Scalars h = x->read_scalars();
  if (h.err & 2) fail(SSCF_E_CAPACITY, "more than %d rotation candidates share the cut-off |F|", MAX_TIES);
  double E = h.e_band + h.e_coul;
  std::memcpy(&info.dq_max, &h.dq_bits, sizeof(double));
  std::memcpy(&info.max_abs_fov, &h.fov_bits, sizeof(double));
  info.n_candidates = h.n_cand;
  info.n_rotations = h.n_rot;
  info.delta_e = E - E_prev;
  info.converged = (x->criterion == SSCF_CONV_CHARGE) ? (info.dq_max < x->dq_conv)
                                                      : (std::fabs(info.delta_e) < x->e_conv);
  if (info.converged) {
    // occupied-only orthonormalization after convergence (section 4.1)
    double eta2 = 0.0;
    int conv2 = 0;
    x->orthonormalize(1, x->max_sweeps_step, &eta2, &conv2);
    info.post_ortho = 1;
    x->charges(0);
    x->energy_terms();
    h = x->read_scalars();
    E = h.e_band + h.e_coul;
  }
  HIPC(hipEventRecord(x->ev[7], s));
  x->sync();
  info.energy = E;
  info.e_band = h.e_band;
  info.e_coul = h.e_coul;
  info.nnz_tiles = x->active_tiles();
  info.nnz_c = x->count ? x->count_nnz_c() : -1;
  x->counting = false;
  float t[7];
  for (int i = 0; i < 7; ++i) HIPC(hipEventElapsedTime(&t[i], x->ev[i], x->ev[i + 1]));
  info.ms_fock = t[0];
  info.ms_cfc = t[1];
  info.ms_select = t[2];
  info.ms_rot = t[3];
  info.ms_ortho = t[4];
  info.ms_sums = t[5] + t[6];
  HIPC(hipEventElapsedTime(&info.ms_total, x->ev[0], x->ev[7]));
  x->E = E;
  x->pcollect();
  if (out) *out = info;
}

// =========================================================================================
// C ABI
// =========================================================================================

template <class Fn>
static sscf_status guarded(sscf_ctx* x, Fn&& fn) {
  try {
    fn();
  } catch (const Fail& f) {
    x->counting = false;
    x->err = f.msg;
    // the state is not a complete step any more after a runtime or capacity failure
    if (f.code == SSCF_E_HIP || f.code == SSCF_E_CAPACITY) x->failed = true;
    return f.code;
  } catch (const std::exception& e) {
    x->err = e.what();
    return SSCF_E_NOMEM;
  }
  return SSCF_OK;
}

extern "C" {

sscf_status sscf_init_system(const sscf_system_desc* desc, sscf_ctx** out) {
  if (!out) { g_init_error = "out is NULL"; return SSCF_E_INVALID_ARG; }
  *out = nullptr;
  sscf_ctx* x = nullptr;
  try {
    x = new sscf_ctx();
    build(x, desc);
  } catch (const Fail& f) {
    g_init_error = f.msg;
    if (x) { x->release(); delete x; }
    return f.code;
  } catch (const std::exception& e) {
    g_init_error = e.what();
    if (x) { x->release(); delete x; }
    return SSCF_E_NOMEM;
  }
  g_init_error.clear();
  *out = x;
  return SSCF_OK;
}

sscf_status sscf_set_fock(sscf_ctx* x, const double* f_val, int32_t mode) {
  if (!x) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    if (x->failed) fail(SSCF_E_STATE, "context failed earlier: %s", x->err.c_str());
    if (!f_val || (mode != SSCF_FOCK_H0 && mode != SSCF_FOCK_FULL)) fail(SSCF_E_INVALID_ARG, "bad set_fock arguments");
    for (int64_t t = 0; t < x->n_val; ++t)
      if (!std::isfinite(f_val[t])) fail(SSCF_E_INVALID_ARG, "non-finite Fock value at %lld", (long long)t);
    const auto& rp = x->h_blk_rowptr;
    const auto& col = x->h_blk_col;
    for (int a = 0; a < x->v.n_atoms; ++a)
      for (int64_t k = rp[a]; k < rp[a + 1]; ++k) {
        const int b = col[k];
        const int64_t kt = std::lower_bound(col.begin() + rp[b], col.begin() + rp[b + 1], a) - col.begin();
        const int nA = x->h_atom_nao[a], nB = x->h_atom_nao[b];
        for (int i = 0; i < nA; ++i)
          for (int j = 0; j < nB; ++j)
            if (f_val[x->h_blk_off[k] + (int64_t)i * nB + j] != f_val[x->h_blk_off[kt] + (int64_t)j * nA + i])
              fail(SSCF_E_INVALID_ARG, "Fock matrix is not symmetric (atoms %d, %d)", a, b);
      }
    const size_t nxe = (size_t)x->v.nbx * 256;
    double* tmp = x->upload(f_val, x->n_val);
    double* dst = (mode == SSCF_FOCK_H0) ? x->H0 : (x->Hfull ? x->Hfull : (x->Hfull = x->dalloc<double>(nxe)));
    HIPC(hipMemsetAsync(dst, 0, nxe * sizeof(double), x->stream));
    launch_scatter(x->val_map, x->n_val, tmp, dst, x->stream);
    x->dfree(tmp);
    x->fock_full = (mode == SSCF_FOCK_FULL);
    x->sync();
  });
}

sscf_status sscf_scf_step(sscf_ctx* x, sscf_step_info* info) {
  if (!x) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    if (x->failed) fail(SSCF_E_STATE, "context failed earlier: %s", x->err.c_str());
    step(x, info);
  });
}

sscf_status sscf_fragment_guess(const sscf_guess_desc* d, int64_t* c0_colptr, int32_t* c0_row, double* c0_val,
                                int64_t cap, int32_t* mo_group, int64_t* nnz, int32_t* n_occ) {
  if (!d || !nnz || !n_occ) return SSCF_E_INVALID_ARG;
  std::vector<void*> mem;
  auto freeall = [&] { for (void* m : mem) hipFree(m); mem.clear(); };
  try {
    const int na = d->n_atoms, nf = d->n_frag;
    if (na <= 0 || nf <= 0 || d->n_groups <= 0 || !d->atom_nao || !d->blk_rowptr || !d->blk_col || !d->blk_off ||
        !d->S_val || !d->H0_val || !d->atom_frag || !d->frag_nocc || !d->frag_group || !(d->drop >= 0.0))
      fail(SSCF_E_INVALID_ARG, "guess: missing arrays or bad sizes");
    std::vector<int64_t> ao_off(na + 1, 0);
    for (int a = 0; a < na; ++a) {
      if (d->atom_nao[a] < 1) fail(SSCF_E_INVALID_ARG, "guess: atom %d has no AO", a);
      ao_off[a + 1] = ao_off[a] + d->atom_nao[a];
    }
    std::vector<int> atom0(nf + 1, -1);
    for (int a = 0; a < na; ++a) {
      const int f = d->atom_frag[a];
      if (f < 0 || f >= nf || (a > 0 && f < d->atom_frag[a - 1]) || (a > 0 && f > d->atom_frag[a - 1] + 1) ||
          (a == 0 && f != 0))
        fail(SSCF_E_INVALID_ARG, "guess: atom_frag must run 0, 0, .., 1, .. over the atoms");
      if (atom0[f] < 0) atom0[f] = a;
    }
    if (d->atom_frag[na - 1] != nf - 1) fail(SSCF_E_INVALID_ARG, "guess: n_frag does not match atom_frag");
    atom0[nf] = na;
    std::vector<int64_t> coff(nf + 1, 0);
    int64_t n_mo = ao_off[na];
    int nocc_total = 0;
    for (int f = 0; f < nf; ++f) {
      const int64_t n = ao_off[atom0[f + 1]] - ao_off[atom0[f]];
      if (n > GUESS_MAXN) fail(SSCF_E_INVALID_ARG, "guess: fragment %d has %lld AOs (at most %d)", f, (long long)n, GUESS_MAXN);
      if (d->frag_nocc[f] < 0 || d->frag_nocc[f] > n) fail(SSCF_E_INVALID_ARG, "guess: fragment %d: bad frag_nocc", f);
      if (d->frag_group[f] < 0 || d->frag_group[f] >= d->n_groups) fail(SSCF_E_INVALID_ARG, "guess: fragment %d: bad group", f);
      coff[f + 1] = coff[f] + n * n;
      nocc_total += d->frag_nocc[f];
    }
    const int64_t nblk = d->blk_rowptr[na];
    if (d->blk_rowptr[0] != 0 || nblk <= 0 || d->n_val <= 0) fail(SSCF_E_INVALID_ARG, "guess: empty or bad pattern");
    for (int a = 0; a < na; ++a) {
      if (d->blk_rowptr[a + 1] < d->blk_rowptr[a]) fail(SSCF_E_INVALID_ARG, "guess: bad blk_rowptr");
      for (int64_t k = d->blk_rowptr[a]; k < d->blk_rowptr[a + 1]; ++k) {
        const int b = d->blk_col[k];
        if (b < 0 || b >= na) fail(SSCF_E_INVALID_ARG, "guess: bad blk_col");
        if (d->blk_off[k] < 0 || d->blk_off[k] + (int64_t)d->atom_nao[a] * d->atom_nao[b] > d->n_val)
          fail(SSCF_E_INVALID_ARG, "guess: block %lld lies outside the %lld values", (long long)k, (long long)d->n_val);
      }
    }
    for (int64_t k = 0; k < d->n_val; ++k)
      if (!std::isfinite(d->S_val[k]) || !std::isfinite(d->H0_val[k])) fail(SSCF_E_INVALID_ARG, "guess: non-finite value");
    hipStream_t s = (hipStream_t)d->hip_stream;
    auto up = [&](const void* src, size_t bytes) {
      void* p = nullptr;
      HIPC(hipMalloc(&p, bytes ? bytes : 1));
      mem.push_back(p);
      if (src && bytes) HIPC(hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, s));
      return p;
    };
    auto* datom0 = (int*)up(atom0.data(), sizeof(int) * (nf + 1));
    auto* daoo = (int64_t*)up(ao_off.data(), sizeof(int64_t) * (na + 1));
    auto* drp = (int64_t*)up(d->blk_rowptr, sizeof(int64_t) * (na + 1));
    auto* dbc = (int*)up(d->blk_col, sizeof(int) * nblk);
    auto* dbo = (int64_t*)up(d->blk_off, sizeof(int64_t) * nblk);
    auto* dnao = (int*)up(d->atom_nao, sizeof(int) * na);
    auto* dS = (double*)up(d->S_val, sizeof(double) * d->n_val);
    auto* dH = (double*)up(d->H0_val, sizeof(double) * d->n_val);
    auto* dco = (int64_t*)up(coff.data(), sizeof(int64_t) * (nf + 1));
    auto* dout = (double*)up(nullptr, sizeof(double) * coff[nf]);
    auto* dlam = (double*)up(nullptr, sizeof(double) * n_mo);
    int zero = 0;
    auto* derr = (int*)up(&zero, sizeof(int));
    launch_fragment_guess(nf, datom0, daoo, drp, dbc, dbo, dnao, dS, dH, dco, dout, dlam, derr, s);
    std::vector<double> out(coff[nf]);
    int err = 0;
    HIPC(hipMemcpyAsync(out.data(), dout, sizeof(double) * coff[nf], hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(&err, derr, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    freeall();
    if (err & 1) fail(SSCF_E_NOT_SPD, "guess: a fragment's overlap block is not positive definite");
    // columns: occupied of group 0, 1, .., then virtual; fragments ascending in a group
    std::vector<std::vector<int>> frags(d->n_groups);
    for (int f = 0; f < nf; ++f) frags[d->frag_group[f]].push_back(f);
    int64_t count = 0;
    std::vector<std::array<int64_t, 3>> cols;   // (fragment, local MO, nonzeros)
    cols.reserve(n_mo);
    for (int pass = 0; pass < 2; ++pass)
      for (int g = 0; g < d->n_groups; ++g)
        for (int f : frags[g]) {
          const int n = (int)(ao_off[atom0[f + 1]] - ao_off[atom0[f]]);
          const int j0 = pass == 0 ? 0 : d->frag_nocc[f], j1 = pass == 0 ? d->frag_nocc[f] : n;
          for (int j = j0; j < j1; ++j) {
            int64_t c = 0;
            for (int i = 0; i < n; ++i) c += std::fabs(out[coff[f] + (int64_t)i * n + j]) >= d->drop;
            cols.push_back({f, j, c});
            count += c;
          }
        }
    *nnz = count;
    *n_occ = nocc_total;
    if (count > cap || !c0_colptr || !c0_row || !c0_val || !mo_group)
      fail(SSCF_E_CAPACITY, "guess: %lld coefficients do not fit in cap %lld", (long long)count, (long long)cap);
    c0_colptr[0] = 0;
    for (size_t col = 0; col < cols.size(); ++col) {
      const int f = (int)cols[col][0], j = (int)cols[col][1];
      const int n = (int)(ao_off[atom0[f + 1]] - ao_off[atom0[f]]);
      int64_t w = c0_colptr[col];
      for (int i = 0; i < n; ++i) {
        const double v = out[coff[f] + (int64_t)i * n + j];
        if (std::fabs(v) >= d->drop) { c0_row[w] = (int32_t)(ao_off[atom0[f]] + i); c0_val[w] = v; ++w; }
      }
      c0_colptr[col + 1] = w;
      mo_group[col] = d->frag_group[f];
    }
    return SSCF_OK;
  } catch (const Fail& f) {
    freeall();
    g_init_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    freeall();
    g_init_error = e.what();
    return SSCF_E_NOMEM;
  }
}

sscf_status sscf_atom_neighbours(int32_t n_atoms, const double* xyz, double cutoff, void* hip_stream,
                                 int64_t* rowptr, int32_t* col, int64_t cap, int64_t* nnz) {
  if (!xyz || !nnz) {
    g_init_error = "atom neighbours: NULL argument";
    return SSCF_E_INVALID_ARG;
  }
  std::vector<void*> mem;
  auto freeall = [&] { for (void* m : mem) hipFree(m); mem.clear(); };
  try {
    const int n = n_atoms;
    if (n <= 0) fail(SSCF_E_INVALID_ARG, "atom neighbours: n_atoms must be positive");
    if (!(cutoff > 0.0) || !(cutoff <= 1e100)) fail(SSCF_E_INVALID_ARG, "atom neighbours: cutoff must be in (0, 1e100]");
    for (int64_t i = 0; i < 3LL * n; ++i)
      if (!std::isfinite(xyz[i]) || std::fabs(xyz[i]) > 1e100) fail(SSCF_E_INVALID_ARG, "atom neighbours: bad coordinate");
    hipStream_t s = (hipStream_t)hip_stream;
    auto alloc = [&](size_t bytes) {
      void* p = nullptr;
      HIPC(hipMalloc(&p, bytes ? bytes : 1));
      mem.push_back(p);
      return p;
    };
    const int nt = (n + 63) / 64;
    auto* dxyz = (double*)alloc(sizeof(double) * 3 * n);
    auto* box = (double*)alloc(sizeof(double) * 6 * nt);
    auto* cnt = (int*)alloc(sizeof(int) * n);
    auto* drp = (int64_t*)alloc(sizeof(int64_t) * (n + 1));
    HIPC(hipMemcpyAsync(dxyz, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    launch_atom_nbr_count(n, dxyz, cutoff, box, cnt, drp, s);
    int64_t total = 0;
    HIPC(hipMemcpyAsync(&total, drp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    *nnz = total;
    if (total > cap || !rowptr || !col)
      fail(SSCF_E_CAPACITY, "atom neighbours: %lld entries do not fit in cap %lld", (long long)total, (long long)cap);
    auto* dcol = (int*)alloc(sizeof(int) * total);
    launch_atom_nbr_fill(n, dxyz, cutoff, box, drp, dcol, s);
    HIPC(hipMemcpyAsync(rowptr, drp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(col, dcol, sizeof(int) * total, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    freeall();
    return SSCF_OK;
  } catch (const Fail& f) {
    freeall();
    g_init_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    freeall();
    g_init_error = e.what();
    return SSCF_E_NOMEM;
  }
}

// ---- the atom neighbour map without allocation -------------------------------------------
// Its scratch lives in `scratch`, a fixed array of every GPU the library runs on: the bounding
// boxes of the 64-atom tiles (6 doubles each), the neighbour count of every atom, and an error
// flag.  Host code never passes `scratch` itself (that name is a host-side stand-in): the
// device address of each GPU's copy comes from hipGetSymbolAddress, once per device.
namespace {
constexpr int NOALLOC_TILES = (SSCF_NOALLOC_MAX_ATOMS + NB_TILE_ATOMS - 1) / NB_TILE_ATOMS;
constexpr size_t NOALLOC_BOX = 0;                                                   // doubles
constexpr size_t NOALLOC_CNT = NOALLOC_BOX + sizeof(double) * 6 * NOALLOC_TILES;     // ints
constexpr size_t NOALLOC_FLAG = NOALLOC_CNT + sizeof(int) * SSCF_NOALLOC_MAX_ATOMS;  // one int
constexpr size_t NOALLOC_BYTES = NOALLOC_FLAG + 256;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// device address of this device's scratch (looked up on the first call on the device)
static unsigned char* scratch_of_current_device() {
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) fail(SSCF_E_CAPACITY, "device %d: at most %d devices", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  return g_scratch_ptr[dev];
}

static bool is_device_memory(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}

sscf_status sscf_atom_neighbours_noalloc(int32_t n_atoms, const double* xyz, double cutoff, void* hip_stream,
                                         int64_t* rowptr, int32_t* col, int64_t cap, int64_t* nnz) {
  if (!xyz || !rowptr || !nnz) {
    g_init_error = "atom neighbours (no allocation): NULL argument";
    return SSCF_E_INVALID_ARG;
  }
  try {
    const int n = n_atoms;
    if (n <= 0) fail(SSCF_E_INVALID_ARG, "atom neighbours (no allocation): n_atoms must be positive");
    if (n > SSCF_NOALLOC_MAX_ATOMS)
      fail(SSCF_E_CAPACITY, "atom neighbours (no allocation): %d atoms exceed the fixed scratch's %d", n,
           SSCF_NOALLOC_MAX_ATOMS);
    if (!(cutoff > 0.0) || !(cutoff <= 1e100))
      fail(SSCF_E_INVALID_ARG, "atom neighbours (no allocation): cutoff must be in (0, 1e100]");
    if (!is_device_memory(xyz) || !is_device_memory(rowptr) || (col && !is_device_memory(col)))
      fail(SSCF_E_INVALID_ARG, "atom neighbours (no allocation): xyz, rowptr and col must be device memory");
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned char* base = scratch_of_current_device();
    double* box = reinterpret_cast<double*>(base + NOALLOC_BOX);
    int* cnt = reinterpret_cast<int*>(base + NOALLOC_CNT);
    int* flag = reinterpret_cast<int*>(base + NOALLOC_FLAG);
    // the flag keeps the last call's value: cleared by a kernel (no memset node)
    launch_fill_i32(flag, 1, 0, s);
    launch_check_coords(3LL * n, xyz, flag, s);
    launch_atom_nbr_count(n, xyz, cutoff, box, cnt, rowptr, s);
    int bad = 0;
    int64_t total = 0;
    HIPC(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(&total, rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (bad) fail(SSCF_E_INVALID_ARG, "atom neighbours (no allocation): bad coordinate");
    *nnz = total;
    if (total > cap || !col)
      fail(SSCF_E_CAPACITY, "atom neighbours (no allocation): %lld entries do not fit in cap %lld",
           (long long)total, (long long)cap);
    launch_atom_nbr_fill(n, xyz, cutoff, box, rowptr, col, s);
    // the scratch is free again once the call returns
    HIPC(hipStreamSynchronize(s));
    return SSCF_OK;
  } catch (const Fail& f) {
    g_init_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    g_init_error = e.what();
    return SSCF_E_NOMEM;
  }
}

sscf_status sscf_constrained_kmeans(const sscf_kmeans_desc* d, int32_t* group, double* means_out,
                                    sscf_kmeans_info* info) {
  if (!d || !group || !means_out) {
    g_init_error = "kmeans: NULL argument";
    return SSCF_E_INVALID_ARG;
  }
  std::vector<void*> mem;
  hipStream_t own = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto freeall = [&] {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    if (own) hipStreamSynchronize(own);
    for (void* m : mem) hipFree(m);
    mem.clear();
    if (own) hipStreamDestroy(own);
    own = nullptr;
  };
  try {
    const int n = d->n_points, m = d->n_means, nl = d->n_link;
    if (n <= 0 || m <= 0 || nl <= 0 || !d->points || !d->means0)
      fail(SSCF_E_INVALID_ARG, "kmeans: need n_points, n_means, n_link > 0 and both coordinate arrays");
    if (nl > KM_MAX_LINK) fail(SSCF_E_INVALID_ARG, "kmeans: n_link %d exceeds %d", nl, KM_MAX_LINK);
    if (m > KM_MAX_MEANS) fail(SSCF_E_INVALID_ARG, "kmeans: %d means exceed %d", m, KM_MAX_MEANS);
    if ((int64_t)m * nl < n)
      fail(SSCF_E_INVALID_ARG, "kmeans: %d means of at most %d points cannot hold %d points", m, nl, n);
    if (d->max_iter < 1 || !(d->tol >= 0.0) || !std::isfinite(d->tol))
      fail(SSCF_E_INVALID_ARG, "kmeans: max_iter >= 1 and a finite tol >= 0 are required");
    for (int64_t i = 0; i < 3LL * n; ++i)
      if (!std::isfinite(d->points[i]) || std::fabs(d->points[i]) > 1e100) fail(SSCF_E_INVALID_ARG, "kmeans: bad point coordinate");
    for (int64_t i = 0; i < 3LL * m; ++i)
      if (!std::isfinite(d->means0[i]) || std::fabs(d->means0[i]) > 1e100) fail(SSCF_E_INVALID_ARG, "kmeans: bad mean coordinate");
    // the rounds are replayed from a captured graph, which needs a stream other than the
    // legacy default one: without a caller's stream the work goes to a stream of its own
    hipStream_t s = (hipStream_t)d->hip_stream;
    if (!s) {
      HIPC(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
      s = own;
    }
    auto alloc = [&](size_t bytes) {
      void* p = nullptr;
      HIPC(hipMalloc(&p, bytes ? bytes : 1));
      mem.push_back(p);
      return p;
    };
    auto* pts = (double*)alloc(sizeof(double) * 3 * n);
    auto* ma = (double*)alloc(sizeof(double) * 3 * m);     // current means (fixed: the graph reads it)
    auto* mb = (double*)alloc(sizeof(double) * 3 * m);     // moved means
    auto* rank = (int*)alloc(sizeof(int) * (size_t)n * m);
    auto* assign = (int*)alloc(sizeof(int) * n);
    auto* next = (int*)alloc(sizeof(int) * n);
    auto* prop = (int*)alloc(sizeof(int) * n);
    auto* held = (int*)alloc(sizeof(int) * (size_t)m * nl);
    auto* n_held = (int*)alloc(sizeof(int) * m);
    auto* pcnt = (int*)alloc(sizeof(int) * m);
    auto* plist = (int*)alloc(sizeof(int) * (size_t)m * KM_PCAP);
    constexpr int BATCH = 8;                 // rounds between two looks at the free counts
    auto* n_free = (int*)alloc(sizeof(int) * BATCH);
    auto* disp = (double*)alloc(sizeof(double));
    HIPC(hipMemcpyAsync(pts, d->points, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    HIPC(hipMemcpyAsync(ma, d->means0, sizeof(double) * 3 * m, hipMemcpyHostToDevice, s));
    // every round that turns a point away advances that point's next[] by one, and next
    // stays below m (the means hold m * n_link >= n points), so the rounds of one
    // attribution are at most n * (m - 1) + 1
    const int64_t max_rounds = (int64_t)n * (m - 1) + 1;
    // one batch of rounds, captured once and replayed: the rounds are short and launch-bound
    HIPC(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int b = 0; b < BATCH; ++b)
      launch_km_round(n, m, nl, pts, ma, rank, assign, next, prop, pcnt, plist, held, n_held, n_free + b, s);
    HIPC(hipStreamEndCapture(s, &graph));
    HIPC(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    int it = 0;
    int64_t rounds_total = 0;
    double dsum = 0.0;
    for (it = 0; it < d->max_iter;) {
      launch_km_rank(n, m, pts, ma, rank, s);
      launch_km_reset(n, m, assign, next, n_held, pcnt, s);
      int64_t r = 0;
      bool placed = false;
      while (!placed) {
        HIPC(hipGraphLaunch(exec, s));
        int nf[BATCH];
        HIPC(hipMemcpyAsync(nf, n_free, sizeof(nf), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        for (int b = 0; b < BATCH && !placed; ++b) {
          ++r;
          placed = nf[b] == 0;
        }
        if (!placed && r > max_rounds) fail(SSCF_E_HIP, "kmeans: attribution did not settle in %lld rounds", (long long)r);
      }
      rounds_total += r;
      launch_km_move(n, m, pts, assign, ma, mb, disp, s);
      HIPC(hipMemcpyAsync(ma, mb, sizeof(double) * 3 * m, hipMemcpyDeviceToDevice, s));
      HIPC(hipMemcpyAsync(&dsum, disp, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      ++it;
      if (dsum / m < d->tol) break;
    }
    HIPC(hipMemcpyAsync(group, assign, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(means_out, ma, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    freeall();
    if (info) {
      info->iterations = it;
      info->rounds = rounds_total;
      info->displacement = dsum / m;
    }
    return SSCF_OK;
  } catch (const Fail& f) {
    freeall();
    g_init_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    freeall();
    g_init_error = e.what();
    return SSCF_E_NOMEM;
  }
}

sscf_status sscf_set_control(sscf_ctx* x, const sscf_control* c) {
  if (!x || !c) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    if (!(c->eps >= 0.0) || !std::isfinite(c->eps) || !(c->e_conv >= 0.0) || !std::isfinite(c->e_conv) ||
        !(c->dq_conv >= 0.0) || !std::isfinite(c->dq_conv))
      fail(SSCF_E_INVALID_ARG, "thresholds must be finite and non-negative");
    if (c->criterion != SSCF_CONV_ENERGY && c->criterion != SSCF_CONV_CHARGE)
      fail(SSCF_E_INVALID_ARG, "unknown criterion %d", c->criterion);
    if (c->step_ortho != 0 && c->step_ortho != 1) fail(SSCF_E_INVALID_ARG, "step_ortho must be 0 or 1");
    x->eps = c->eps;
    x->e_conv = c->e_conv;
    x->dq_conv = c->dq_conv;
    x->criterion = c->criterion;
    x->step_ortho = c->step_ortho;
  });
}

sscf_status sscf_get_control(const sscf_ctx* x, sscf_control* c) {
  if (!x || !c) return SSCF_E_INVALID_ARG;
  c->eps = x->eps;
  c->e_conv = x->e_conv;
  c->dq_conv = x->dq_conv;
  c->criterion = x->criterion;
  c->step_ortho = x->step_ortho;
  return SSCF_OK;
}

sscf_status sscf_orthonormalize(sscf_ctx* x, int32_t occ_only, sscf_step_info* out) {
  if (!x || (occ_only != 0 && occ_only != 1)) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    if (x->failed) fail(SSCF_E_STATE, "context failed earlier: %s", x->err.c_str());
    sscf_step_info info;
    std::memset(&info, 0, sizeof(info));
    double eta = 0.0;
    int conv = 0;
    x->counting = true;
    const int sweeps = x->orthonormalize(occ_only, x->max_sweeps_init, &eta, &conv);
    if (!conv) fail(SSCF_E_ORTHO, "orthonormalization did not reach eps/100 in %d sweeps (eta %.3e)", sweeps, eta);
    x->charges(0);
    x->energy_terms();
    x->counting = false;
    const Scalars h = x->read_scalars();
    x->E = h.e_band + h.e_coul;
    info.energy = x->E;
    info.e_band = h.e_band;
    info.e_coul = h.e_coul;
    info.n_ortho_sweeps = sweeps;
    info.ortho_eta = eta;
    info.ortho_converged = conv;
    info.nnz_tiles = x->active_tiles();
    info.nnz_c = x->count ? x->count_nnz_c() : -1;
    x->pcollect();
    if (out) *out = info;
  });
}

sscf_status sscf_memory_info(const sscf_ctx* x, size_t* device_bytes, int64_t* tile_slots, int64_t* tile_slots_y,
                             int64_t* tiles) {
  if (!x || !device_bytes || !tile_slots || !tile_slots_y || !tiles) return SSCF_E_INVALID_ARG;
  size_t b = 0;
  for (size_t n : x->owned_bytes) b += n;
  *device_bytes = b;
  *tile_slots = (int64_t)x->n_slots;
  *tile_slots_y = (int64_t)x->n_slots_y;
  *tiles = (int64_t)x->v.G * x->v.n_rb;
  return SSCF_OK;
}

sscf_status sscf_get_energy(const sscf_ctx* x, double* e) {
  if (!x || !e) return SSCF_E_INVALID_ARG;
  *e = x->E;
  return SSCF_OK;
}

sscf_status sscf_init_info(const sscf_ctx* x, sscf_step_info* info) {
  if (!x || !info) return SSCF_E_INVALID_ARG;
  *info = x->init_info;
  return SSCF_OK;
}

sscf_status sscf_get_charges(const sscf_ctx* cx, double* q, size_t n) {
  sscf_ctx* x = const_cast<sscf_ctx*>(cx);
  if (!x || !q || n < (size_t)x->v.n_atoms) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    HIPC(hipMemcpyAsync(q, x->q, sizeof(double) * x->v.n_atoms, hipMemcpyDeviceToHost, x->stream));
    x->sync();
  });
}

sscf_status sscf_get_density(const sscf_ctx* cx, double* p_val, size_t n_val) {
  sscf_ctx* x = const_cast<sscf_ctx*>(cx);
  if (!x || !p_val || n_val < (size_t)x->n_val) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    if (!x->pblk) x->pblk = x->dalloc<double>((size_t)x->v.nbx * 256);
    if (!x->pval) x->pval = x->dalloc<double>(x->n_val);
    launch_list_t(x->v, x->actC[x->cur], x->listT, x->cntT, x->stream);
    launch_density_blocks(x->v, x->C[x->cur], x->cmask[x->cur], x->listT, x->cntT, x->C[x->cur], x->actC[x->cur],
                          x->cmask[x->cur], false, x->pblk, x->stream);
    launch_gather(x->val_map, x->n_val, x->pblk, x->pval, x->stream);
    HIPC(hipMemcpyAsync(p_val, x->pval, sizeof(double) * x->n_val, hipMemcpyDeviceToHost, x->stream));
    x->sync();
  });
}

sscf_status sscf_get_energy_gradient(sscf_ctx* x, double* dE_dX, double* dE_dS, size_t n_val) {
  if (!x || !dE_dX || !dE_dS || n_val < (size_t)x->n_val) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    if (x->failed) fail(SSCF_E_STATE, "context failed earlier: %s", x->err.c_str());
    if (!x->gx) x->gx = x->dalloc<double>(x->n_val);
    if (!x->gs) x->gs = x->dalloc<double>(x->n_val);
    x->gradient(x->gx, x->gs, nullptr);
    HIPC(hipMemcpyAsync(dE_dX, x->gx, sizeof(double) * x->n_val, hipMemcpyDeviceToHost, x->stream));
    HIPC(hipMemcpyAsync(dE_dS, x->gs, sizeof(double) * x->n_val, hipMemcpyDeviceToHost, x->stream));
    x->sync();
  });
}

sscf_status sscf_get_energy_gradient_device(sscf_ctx* x, double* dE_dX, double* dE_dS, size_t n_val,
                                            double* dE_donsite, size_t n_onsite) {
  if (!x || !dE_dX || !dE_dS || n_val < (size_t)x->n_val) return SSCF_E_INVALID_ARG;
  if (dE_donsite && n_onsite < 2 * (size_t)x->v.n_atoms) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    if (x->failed) fail(SSCF_E_STATE, "context failed earlier: %s", x->err.c_str());
    hipPointerAttribute_t at;
    for (double* p : {dE_dX, dE_dS, dE_donsite}) {
      if (!p) continue;
      if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        fail(SSCF_E_INVALID_ARG, "gradient outputs must be device memory");
      }
    }
    x->gradient(dE_dX, dE_dS, dE_donsite);
  });
}

sscf_status sscf_get_mo_coefficients(const sscf_ctx* cx, int64_t* colptr, int32_t* row, double* val, int64_t* nnz) {
  sscf_ctx* x = const_cast<sscf_ctx*>(cx);
  if (!x || !nnz) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    const View& v = x->v;
    const size_t ntiles = (size_t)v.G * v.n_rb;
    std::vector<uint8_t> act(ntiles);
    std::vector<int> hslot(ntiles);
    HIPC(hipMemcpyAsync(act.data(), x->actC[x->cur], ntiles, hipMemcpyDeviceToHost, x->stream));
    HIPC(hipMemcpyAsync(hslot.data(), x->slot, sizeof(int) * ntiles, hipMemcpyDeviceToHost, x->stream));
    x->sync();
    std::vector<std::vector<std::pair<int32_t, double>>> cols(v.n_mo);
    std::vector<double> tile((size_t)RB * v.W);
    for (int g = 0; g < v.G; ++g)
      for (int r = 0; r < v.n_rb; ++r) {
        const size_t t = (size_t)g * v.n_rb + r;
        if (!act[t]) continue;
        HIPC(hipMemcpyAsync(tile.data(), x->C[x->cur] + (size_t)hslot[t] * RB * v.W, sizeof(double) * RB * v.W,
                            hipMemcpyDeviceToHost, x->stream));
        x->sync();
        for (int k = 0; k < RB; ++k)
          for (int c = 0; c < v.W; ++c) {
            const double val_ = tile[(size_t)k * v.W + c];
            const int j = x->h_mo_of[(size_t)g * v.W + c];
            if (val_ != 0.0 && j >= 0) cols[j].push_back({r * RB + k, val_});
          }
      }
    int64_t total = 0;
    for (auto& c : cols) total += (int64_t)c.size();
    if (row && val && colptr) {
      if (*nnz < total) fail(SSCF_E_INVALID_ARG, "buffers too small: %lld entries needed", (long long)total);
      int64_t p = 0;
      colptr[0] = 0;
      for (int j = 0; j < v.n_mo; ++j) {
        for (auto& e : cols[j]) { row[p] = e.first; val[p] = e.second; ++p; }
        colptr[j + 1] = p;
      }
    }
    *nnz = total;
  });
}

sscf_status sscf_get_schedule(const sscf_ctx* x, int32_t* g, int32_t* h, int32_t* round, int32_t* n_blocks) {
  if (!x || !n_blocks) return SSCF_E_INVALID_ARG;
  if (g && h && round) {
    if (*n_blocks < x->n_blocks) return SSCF_E_INVALID_ARG;
    for (int b = 0; b < x->n_blocks; ++b) { g[b] = x->h_jb_g[b]; h[b] = x->h_jb_h[b]; round[b] = x->h_jb_round[b]; }
  }
  *n_blocks = x->n_blocks;
  return SSCF_OK;
}

sscf_status sscf_get_rotations(const sscf_ctx* cx, int32_t* occ, int32_t* virt, int64_t* n) {
  sscf_ctx* x = const_cast<sscf_ctx*>(cx);
  if (!x || !n) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    const View& v = x->v;
    const size_t per = (size_t)v.OW * v.VW;
    std::vector<int> cnt(x->n_blocks);
    HIPC(hipMemcpyAsync(cnt.data(), x->rot_cnt, sizeof(int) * cnt.size(), hipMemcpyDeviceToHost, x->stream));
    x->sync();
    int64_t tot = 0;
    for (int c : cnt) tot += c;
    if (occ && virt) {
      if (*n < tot) fail(SSCF_E_INVALID_ARG, "room for %lld rotations, %lld selected", (long long)*n, (long long)tot);
      std::vector<int2> sl((size_t)x->n_blocks * per);
      std::vector<int> tc((size_t)x->n_blocks * v.W);
      HIPC(hipMemcpyAsync(sl.data(), x->rot_slot, sizeof(int2) * sl.size(), hipMemcpyDeviceToHost, x->stream));
      HIPC(hipMemcpyAsync(tc.data(), x->tcol, sizeof(int) * tc.size(), hipMemcpyDeviceToHost, x->stream));
      x->sync();
      int64_t k = 0;
      for (int b = 0; b < x->n_blocks; ++b) {
        const int g = x->h_jb_g[b], h = x->h_jb_h[b];
        for (int q = 0; q < cnt[b]; ++q) {
          const int2 r = sl[(size_t)b * per + q];
          occ[k] = x->h_mo_of[(size_t)g * v.W + tc[(size_t)b * v.W + r.x]];
          virt[k] = x->h_mo_of[(size_t)h * v.W + tc[(size_t)b * v.W + r.y]];
          ++k;
        }
      }
    }
    *n = tot;
  });
}

sscf_status sscf_get_kernel_stats(const sscf_ctx* cx, sscf_kernel_stat* out, int32_t* n) {
  sscf_ctx* x = const_cast<sscf_ctx*>(cx);
  if (!x || !n) return SSCF_E_INVALID_ARG;
  if (!out) { *n = SSCF_N_KERNEL_CLASSES; return SSCF_OK; }
  if (*n < SSCF_N_KERNEL_CLASSES) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    if (!x->prof && !x->count)
      fail(SSCF_E_STATE, "neither profiling (SSCF_FLAG_PROFILE) nor work counting (SSCF_FLAG_COUNT_WORK) was requested");
    unsigned long long c[SSCF_N_KERNEL_CLASSES];
    HIPC(hipMemcpyAsync(c, x->pctr, sizeof(c), hipMemcpyDeviceToHost, x->stream));
    x->sync();
    for (int k = 0; k < SSCF_N_KERNEL_CLASSES; ++k) {
      std::memset(out[k].name, 0, sizeof(out[k].name));
      std::strncpy(out[k].name, KC_NAME[k], sizeof(out[k].name) - 1);
      out[k].launches = x->plaunch[k];
      out[k].ms = x->pms[k];
      out[k].mfma_flops = KC_FLOP_PER_MFMA * (double)c[k];
      out[k].alg_flops = x->count ? x->wfl[k] : -1.0;
      out[k].alg_bytes = x->count ? x->wby[k] : -1.0;
    }
    *n = SSCF_N_KERNEL_CLASSES;
  });
}

sscf_status sscf_reset_kernel_stats(sscf_ctx* x) {
  if (!x) return SSCF_E_INVALID_ARG;
  return guarded(x, [&] {
    if (!x->prof && !x->count)
      fail(SSCF_E_STATE, "neither profiling (SSCF_FLAG_PROFILE) nor work counting (SSCF_FLAG_COUNT_WORK) was requested");
    x->pcollect();
    for (int k = 0; k < SSCF_N_KERNEL_CLASSES; ++k) { x->pms[k] = 0.0; x->plaunch[k] = 0; x->wfl[k] = 0.0; x->wby[k] = 0.0; }
    HIPC(hipMemsetAsync(x->pctr, 0, sizeof(unsigned long long) * SSCF_N_KERNEL_CLASSES, x->stream));
    x->sync();
  });
}

void sscf_destroy(sscf_ctx* x) {
  if (!x) return;
  x->release();
  delete x;
}

const char* sscf_last_error(const sscf_ctx* x) {
  if (!x) return g_init_error.c_str();
  return x->err.c_str();
}

}  // extern "C"
