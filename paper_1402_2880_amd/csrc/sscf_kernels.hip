// HIP kernels of the sparse SCF hot path for gfx950 (MI355X, wave64).
//
// Paper: A. Scemama, N. Renon, M. Rapacioli, "A Sparse SCF algorithm and its
// parallel implementation: Application to DFTB", arXiv:1402.2880.
//
// The C^T X C products of section 3.6 (X = S for the orthonormalization,
// X = H for the partial diagonalization) run as block-sparse products of dense
// 16-row tiles on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  The pair
// combinations of section 3.4 are the product C D_sel on the same tiles.  The
// Jacobi rotations of section 3.5 are composed per block into small orthogonal
// matrices and applied in one pass over row blocks, since rows of C are
// independent under right multiplication.  The energy gradient reuses these
// products plus C_occ F (k_apply_occ).  The set-up kernels of sections 3.2 and 3.3
// live in sscf_setup.hip.
//
// FP64 16x16x4 MFMA operand layout (lane l of the wave): A[l % 16][l / 16],
// B[l / 16][l % 16]; result register r holds D[l / 16 + 4 r][l % 16].
#include "sscf_internal.h"

#include <math.h>

namespace sscf {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// block-wide max of a non-negative double, folded into *bits with atomicMax
__device__ void block_max_to(double v, unsigned long long* bits) {
  __shared__ double red[16];
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, red[i]);
    atomicMax(bits, dbits(m));
  }
}

static inline unsigned int nblk(size_t n, int t) { return (unsigned int)((n + t - 1) / t); }

// ---------------------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------------------

__global__ void k_fill(double* p, size_t n, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u8(uint8_t* p, size_t n, uint8_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_i32(int* p, size_t n, int v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

void launch_fill(double* p, size_t n, double v, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256) < 65536 ? nblk(n, 256) : 65536), dim3(256), 0, s, p, n, v);
}
void launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_u8, dim3(nblk(n, 256) < 65536 ? nblk(n, 256) : 65536), dim3(256), 0, s, p, n, v);
}
void launch_fill_i32(int* p, size_t n, int v, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, 256) < 65536 ? nblk(n, 256) : 65536), dim3(256), 0, s, p, n, v);
}

__global__ void k_gather(const int64_t* map, int64_t n, const double* src, double* dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[map[i]];
}
__global__ void k_scatter(const int64_t* map, int64_t n, const double* src, double* dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[map[i]] = src[i];
}
void launch_gather(const int64_t* map, int64_t n, const double* src, double* dst, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_gather, dim3(nblk(n, 256)), dim3(256), 0, s, map, n, src, dst);
}
void launch_scatter(const int64_t* map, int64_t n, const double* src, double* dst, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_scatter, dim3(nblk(n, 256)), dim3(256), 0, s, map, n, src, dst);
}

// a nonzero of C fell on tile (g, r) = tile, which has no slot: the first such tile (+ 1) is
// kept for the error report
__device__ __forceinline__ void note_capacity(int* cap_err, size_t tile) {
  atomicCAS(cap_err, 0, tile < (size_t)INT32_MAX - 1 ? (int)tile + 1 : INT32_MAX);
}

// C0 (one entry per thread) into the tiles
__global__ void k_scatter_c0(int nnz, const int64_t* col_of, const int* row, const double* val,
                             const int* mo_panel, const int* mo_col, int n_rb, int W, const int* slot, double* C,
                             uint8_t* act, unsigned int* cmask, int* cap_err) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int j = (int)col_of[e];
  const int mu = row[e];
  const int g = mo_panel[j];
  const size_t tile = (size_t)g * n_rb + mu / RB;
  const int sl = slot[tile];
  if (sl < 0) {                                 // outside the tile capacity
    note_capacity(cap_err, tile);
    return;
  }
  C[((size_t)sl * RB + (mu % RB)) * W + mo_col[j]] = val[e];
  act[tile] = 1;
  if (val[e] != 0.0) atomicOr(&cmask[tile], 1u << (mo_col[j] >> 4));
}
void launch_scatter_c0(const View& v, int nnz, const int64_t* col_of, const int* row, const double* val,
                       const int* mo_panel, const int* mo_col, double* C, uint8_t* act, unsigned int* cmask,
                       int* cap_err, hipStream_t s) {
  if (nnz) hipLaunchKernelGGL(k_scatter_c0, dim3(nblk(nnz, 256)), dim3(256), 0, s, nnz, col_of, row, val,
                              mo_panel, mo_col, v.n_rb, v.W, v.slot, C, act, cmask, cap_err);
}

// ---------------------------------------------------------------------------------------
// Workgroups go round-robin over the 8 XCDs of the chip, each with its own L2: linear
// workgroup id L runs on XCD L % 8.  Kernels that work group by group decode L so that all
// workgroups of one MO group land on one XCD, in group-major order, and share its L2.
// ---------------------------------------------------------------------------------------

constexpr int N_XCD = 8;

__device__ inline int xcd_group_chunk(int nchunk, int& chunk) {
  const int L = (int)blockIdx.x, slot = L / N_XCD;
  chunk = slot % nchunk;
  return L % N_XCD + N_XCD * (slot / nchunk);
}
static inline unsigned int xcd_grid(int G, int nchunk) {
  return (unsigned int)(N_XCD * ((G + N_XCD - 1) / N_XCD) * nchunk);
}
// Kernels with one wave per listed tile of a group walk the group's list four tiles (one
// workgroup) at a time: workgroup c of the group takes the steps c, c + nchunk, c + 2 nchunk, ...
// The lists live on the device, so the host sizes nchunk from their bound (max_tiles), capped
// so that the launch has about TILE_LIST_WGS workgroups: a grid sized by the bound alone
// would be mostly workgroups with nothing to do where the lists are much shorter than it.
constexpr int TILE_LIST_WGS = 16384;
static inline int tile_list_chunks(int G, int max_tiles) {
  const int need = (max_tiles + 3) / 4;
  const int groups = N_XCD * ((G + N_XCD - 1) / N_XCD);
  const int want = (TILE_LIST_WGS + groups - 1) / groups;
  return std::max(1, std::min(need, want));
}
// item of a list sorted by group, placed by the host on the XCD of its group (-1: padding)
__device__ inline int xcd_item(const int* perm, int maxc) {
  const int L = (int)blockIdx.x;
  return perm[(L % N_XCD) * maxc + L / N_XCD];
}

// ---------------------------------------------------------------------------------------
// supports: dilation of a panel's active row blocks through the pattern of S/H, and the
// sorted lists of active row blocks
// ---------------------------------------------------------------------------------------

// actY[g][r] = 1 where S links row block r to a row block k active in panel g.  The pattern
// of S is symmetric, so the dilation is scattered from the active tiles: one wave per listed
// tile (g, k), its lanes over the row blocks r of row k of the pattern (actY is cleared first).
// A target without a slot is reported (it cannot happen while C keeps to its slots).
__global__ void __launch_bounds__(256) k_dilate(int G, int n_rb, int nchunk, const int* __restrict__ xs_ptr,
                                                const int* __restrict__ xs_col, const int* __restrict__ slotY,
                                                const int* __restrict__ listC, const int* __restrict__ cntC,
                                                uint8_t* __restrict__ actY, int* __restrict__ cap_err) {
  int chunk;
  const int g = xcd_group_chunk(nchunk, chunk);
  if (g >= G) return;
  const int lane = threadIdx.x & 63;
  const size_t gb = (size_t)g * n_rb;
  const int n_t = cntC[g];
  for (int t = chunk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); t < n_t; t += 4 * nchunk) {
    const int k = listC[gb + t];
    for (int e = xs_ptr[k] + lane; e < xs_ptr[k + 1]; e += 64) {
      const size_t idx = gb + xs_col[e];
      if (slotY[idx] < 0)
        note_capacity(cap_err, idx);
      else
        actY[idx] = 1;
    }
  }
}
void launch_dilate(const View& v, const int* listC, const int* cntC, uint8_t* actY, hipStream_t s) {
  launch_fill_u8(actY, (size_t)v.G * v.n_rb, 0, s);
  const int nchunk = tile_list_chunks(v.G, v.max_c);
  hipLaunchKernelGGL(k_dilate, dim3(xcd_grid(v.G, nchunk)), dim3(256), 0, s, v.G, v.n_rb, nchunk, v.xs_ptr, v.xs_col,
                     v.slotY, listC, cntC, actY, v.cap_err);
}

__global__ void __launch_bounds__(256) k_list(int n_rb, const uint8_t* act, int* list, int* cnt) {
  const int g = blockIdx.x;
  __shared__ int wsum[4];
  const uint8_t* a = act + (size_t)g * n_rb;
  int* L = list + (size_t)g * n_rb;
  int base_out = 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int base = 0; base < n_rb; base += 256) {
    const int r = base + threadIdx.x;
    const bool f = r < n_rb && a[r];
    const unsigned long long m = __ballot(f);
    const int pre = __popcll(m & ((1ULL << lane) - 1ULL));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int off = base_out;
    for (int i = 0; i < w; ++i) off += wsum[i];
    if (f) L[off + pre] = r;
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    base_out += tot;
  }
  if (threadIdx.x == 0) cnt[g] = base_out;
}
void launch_list(const View& v, const uint8_t* act, int* list, int* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_list, dim3(v.G), dim3(256), 0, s, v.n_rb, act, list, cnt);
}

// The transposed lists: for row block r, the groups g with act[g][r] set, ascending, in
// listT[r G ...] with their number in cntT[r] (kernels that sum over the groups of a row block
// visit only these, in the order of a loop over all groups)
__global__ void __launch_bounds__(256) k_list_t(int G, int n_rb, const uint8_t* act, int* listT, int* cntT) {
  const int r = blockIdx.x;
  __shared__ int wsum[4];
  int* L = listT + (size_t)r * G;
  int base_out = 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int base = 0; base < G; base += 256) {
    const int g = base + threadIdx.x;
    const bool f = g < G && act[(size_t)g * n_rb + r];
    const unsigned long long m = __ballot(f);
    const int pre = __popcll(m & ((1ULL << lane) - 1ULL));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int off = base_out;
    for (int i = 0; i < w; ++i) off += wsum[i];
    if (f) L[off + pre] = g;
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    base_out += tot;
  }
  if (threadIdx.x == 0) cntT[r] = base_out;
}
void launch_list_t(const View& v, const uint8_t* act, int* listT, int* cntT, hipStream_t s) {
  hipLaunchKernelGGL(k_list_t, dim3(v.n_rb), dim3(256), 0, s, v.G, v.n_rb, act, listT, cntT);
}

// A load that may be known to give zero reads a lane's entry of an all-zero page instead:
// the pointer is selected, the load is unconditional, so every load of a loop body is issued
// before the first wait instead of one at a time behind branches.  The zero buffer holds
// ZCHUNKS chunks of 64 doubles; zl(zp, salt) picks one by a salt that varies between loads,
// so that these reads spread over the L2 channels instead of piling onto one line.
constexpr int ZCHUNKS = ZERO_DOUBLES / 64;
__device__ __forceinline__ const double* zl(const double* zp, unsigned int salt) {
  return zp + ((salt & (ZCHUNKS - 1)) << 6) + (threadIdx.x & 63);
}
__device__ __forceinline__ double ld_or_zero(bool on, const double* p, const double* z) {
  return *(on ? p : z);
}

// ---------------------------------------------------------------------------------------
// out_p = C_g[:, row_off : row_off + 16 MT]^T Y_h[:, col_off : col_off + 16 NT] for pair p = (g, h),
// summed over the row blocks active in both.  Four waves split the MT x NT output tiles 2 x 2.
// ---------------------------------------------------------------------------------------

template <int MW, int NW>
__global__ void __launch_bounds__(256) k_pair(int n_rb, int W, const int* __restrict__ slot,
                                              const int* __restrict__ slotY,
                                              const int* __restrict__ perm, int maxc,
                                              const int* __restrict__ pg,
                                              const int* __restrict__ ph, const double* __restrict__ C,
                                              const int* __restrict__ listC, const int* __restrict__ cntC,
                                              const unsigned int* __restrict__ cmask,
                                              const double* __restrict__ Y, const uint8_t* __restrict__ actY,
                                              const unsigned int* __restrict__ ymask,
                                              int row_off, int MT, int col_off, int NT,
                                              double* __restrict__ out, int ld, size_t out_stride,
                                              unsigned long long* ctr) {
  const int p = xcd_item(perm, maxc);
  if (p < 0) return;
  const int g = pg[p], h = ph[p];
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int MH = (MT + 1) / 2, NH = (NT + 1) / 2;
  const int mt0 = (w >> 1) * MH, nt0 = (w & 1) * NH;
  const int mc = min(MH, MT - mt0), nc = min(NH, NT - nt0);
  d4 acc[MW][NW];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  const size_t gb = (size_t)g * n_rb, hb = (size_t)h * n_rb;
  const int cnt = cntC[g];
  unsigned int n_mfma = 0;
  if (mc > 0 && nc > 0) {
    const unsigned int mcm = (1u << mc) - 1u, ncm = (1u << nc) - 1u;
    const int sa = row_off / 16 + mt0, sb = col_off / 16 + nt0;
    // the rows active in both panels, 64 at a time, with their slice masks, before any product
    for (int base = 0; base < cnt; base += 64) {
      const int t = base + lane;
      int rr = 0, sc = 0, sy = 0;
      unsigned int mab = 0u;
      if (t < cnt) {
        rr = listC[gb + t];
        if (actY[hb + rr]) {
          const unsigned int ma = (cmask[gb + rr] >> sa) & mcm, mb = (ymask[hb + rr] >> sb) & ncm;
          if (ma && mb) {
            mab = ma | (mb << 16);
            sc = slot[gb + rr];                // the common rows' slots in one round trip
            sy = slotY[hb + rr];
          }
        }
      }
      unsigned long long m = __ballot(mab != 0u);
      while (m) {
        const int j = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const unsigned int mj = __builtin_amdgcn_readfirstlane(__shfl((int)mab, j));
        const unsigned int ma = mj & 0xffffu, mb = mj >> 16;
        const size_t scj = (size_t)(unsigned int)__builtin_amdgcn_readfirstlane(__shfl(sc, j));
        const size_t syj = (size_t)(unsigned int)__builtin_amdgcn_readfirstlane(__shfl(sy, j));
        const double* Ct = C + scj * (RB * W) + row_off + mt0 * 16 + lr;
        const double* Yt = Y + syj * (RB * W) + col_off + nt0 * 16 + lr;
        double a[4][MW], b[4][NW];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int ro = (4 * s + lk) * W;
#pragma unroll
          for (int i = 0; i < MW; ++i) a[s][i] = (ma & (1u << i)) ? Ct[ro + i * 16] : 0.0;
#pragma unroll
          for (int jj = 0; jj < NW; ++jj) b[s][jj] = (mb & (1u << jj)) ? Yt[ro + jj * 16] : 0.0;
        }
        // a k-step (4 rows) of a slice that is all zero on either side adds exact zeros
        unsigned int za = 0u, zb = 0u;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
          for (int i = 0; i < MW; ++i)
            if (__ballot(a[s][i] != 0.0)) za |= 1u << (s * MW + i);
#pragma unroll
          for (int jj = 0; jj < NW; ++jj)
            if (__ballot(b[s][jj] != 0.0)) zb |= 1u << (s * NW + jj);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int i = 0; i < MW; ++i)
#pragma unroll
            for (int jj = 0; jj < NW; ++jj)
              if (((za >> (s * MW + i)) & 1u) && ((zb >> (s * NW + jj)) & 1u)) {
                acc[i][jj] = mfma64(a[s][i], b[s][jj], acc[i][jj]);
                ++n_mfma;
              }
      }
    }
  }
  double* o = out + (size_t)p * out_stride;
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j)
      if (i < mc && j < nc)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          o[(size_t)((mt0 + i) * 16 + lk + 4 * q) * ld + (nt0 + j) * 16 + lr] = acc[i][j][q];
  if (ctr && lane == 0 && n_mfma) atomicAdd(ctr, (unsigned long long)n_mfma);
}

void launch_pair(const View& v, int n_pairs, const int* perm, int maxc, const int* pg, const int* ph,
                 const double* C, const int* listC,
                 const int* cntC, const unsigned int* cmask, const double* Y, const uint8_t* actY,
                 const unsigned int* ymask, int row_off, int MT, int col_off, int NT, double* out, int ld,
                 size_t out_stride, unsigned long long* ctr, hipStream_t s) {
  if (n_pairs <= 0) return;
  const int mw = (MT + 1) / 2, nw = (NT + 1) / 2;
  const int m = mw > nw ? mw : nw;
  dim3 grid(N_XCD * maxc), blk(256);
  if (m <= 1)
    hipLaunchKernelGGL((k_pair<1, 1>), grid, blk, 0, s, v.n_rb, v.W, v.slot, v.slotY, perm, maxc, pg, ph, C, listC, cntC, cmask, Y, actY, ymask, row_off, MT, col_off, NT, out, ld, out_stride, ctr);
  else if (m <= 2)
    hipLaunchKernelGGL((k_pair<2, 2>), grid, blk, 0, s, v.n_rb, v.W, v.slot, v.slotY, perm, maxc, pg, ph, C, listC, cntC, cmask, Y, actY, ymask, row_off, MT, col_off, NT, out, ld, out_stride, ctr);
  else if (m <= 3)
    hipLaunchKernelGGL((k_pair<3, 3>), grid, blk, 0, s, v.n_rb, v.W, v.slot, v.slotY, perm, maxc, pg, ph, C, listC, cntC, cmask, Y, actY, ymask, row_off, MT, col_off, NT, out, ld, out_stride, ctr);
  else
    hipLaunchKernelGGL((k_pair<4, 4>), grid, blk, 0, s, v.n_rb, v.W, v.slot, v.slotY, perm, maxc, pg, ph, C, listC, cntC, cmask, Y, actY, ymask, row_off, MT, col_off, NT, out, ld, out_stride, ctr);
}

// per-column dot products d[g][c] = sum_r sum_k C[g][r][k][c] Y[g][r][k][c]
// The active row blocks of panel g are split into CD_SPLIT strided parts, one workgroup each;
// the parts' sums are added in a fixed order by k_coldot_sum.  The workgroup first reads the
// slots and slice masks of up to blockDim.x of its tiles into LDS, one tile per thread, so
// that the walk over them waits on the tiles' values only.

// slots and slice mask of the tiles t0 + stride i (i < n) of panel g, thread i -> LDS entry i
// (mask 0: the tile is skipped); returns the number staged.  Every thread of the block calls it.
__device__ inline int stage_tiles(size_t gb, const int* listC, int t0, int stride, int n, const int* slot,
                                  const int* slotY, const unsigned int* cmask, const uint8_t* actY, int* s_so,
                                  int* s_sy, unsigned int* s_cm) {
  const int i = threadIdx.x;
  unsigned int cm = 0u;
  int so = 0, sy = 0;
  if (i < n) {
    const int r = listC[gb + t0 + stride * i];
    if (actY[gb + r]) {
      cm = cmask[gb + r];
      so = slot[gb + r];
      sy = slotY[gb + r];
    }
  }
  s_cm[i] = cm;
  s_so[i] = so;
  s_sy[i] = sy;
  __syncthreads();
  return n < (int)blockDim.x ? n : (int)blockDim.x;
}

__global__ void __launch_bounds__(256) k_coldot(int n_rb, int W, const int* slot, const int* slotY, const double* C,
                                                const int* listC, const int* cntC, const unsigned int* cmask,
                                                const double* Y, const uint8_t* actY, double* part) {
  __shared__ int s_so[256], s_sy[256];
  __shared__ unsigned int s_cm[256];
  const int g = blockIdx.x, sp = blockIdx.y, c = threadIdx.x;
  const size_t gb = (size_t)g * n_rb;
  const int cnt = cntC[g];
  const int mine = cnt > sp ? (cnt - sp + CD_SPLIT - 1) / CD_SPLIT : 0;   // tiles sp, sp + CD_SPLIT, ...
  double s = 0.0;
  for (int i0 = 0; i0 < mine; i0 += blockDim.x) {
    const int nb = stage_tiles(gb, listC, sp + CD_SPLIT * i0, CD_SPLIT, mine - i0, slot, slotY, cmask, actY, s_so,
                               s_sy, s_cm);
    if (c < W) {
      // two tiles' loads go out together; a zero slice is not read and adds exact zeros, and
      // the terms are added in the same order as one tile at a time
      int j = 0;
      for (; j + 1 < nb; j += 2) {
        const bool on0 = (s_cm[j] >> (c >> 4)) & 1u, on1 = (s_cm[j + 1] >> (c >> 4)) & 1u;
        const double* C0 = C + (size_t)s_so[j] * (RB * W) + c;
        const double* Y0 = Y + (size_t)s_sy[j] * (RB * W) + c;
        const double* C1 = C + (size_t)s_so[j + 1] * (RB * W) + c;
        const double* Y1 = Y + (size_t)s_sy[j + 1] * (RB * W) + c;
        double c0[RB], y0[RB], c1[RB], y1[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
          c0[k] = on0 ? C0[k * W] : 0.0;
          y0[k] = on0 ? Y0[k * W] : 0.0;
          c1[k] = on1 ? C1[k * W] : 0.0;
          y1[k] = on1 ? Y1[k * W] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) s += c0[k] * y0[k];
#pragma unroll
        for (int k = 0; k < RB; ++k) s += c1[k] * y1[k];
      }
      if (j < nb && ((s_cm[j] >> (c >> 4)) & 1u)) {
        const double* Ct = C + (size_t)s_so[j] * (RB * W) + c;
        const double* Yt = Y + (size_t)s_sy[j] * (RB * W) + c;
#pragma unroll
        for (int k = 0; k < RB; ++k) s += Ct[k * W] * Yt[k * W];
      }
    }
    __syncthreads();
  }
  if (c < W) part[((size_t)sp * gridDim.x + g) * W + c] = s;
}
__global__ void k_coldot_sum(size_t n, const double* part, double* out) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int sp = 0; sp < CD_SPLIT; ++sp) s += part[(size_t)sp * n + i];
  out[i] = s;
}
void launch_coldot(const View& v, const double* C, const int* listC, const int* cntC, const unsigned int* cmask,
                   const double* Y, const uint8_t* actY, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_coldot, dim3(v.G, CD_SPLIT), dim3(v.W <= 64 ? 64 : (v.W <= 128 ? 128 : 256)), 0, s, v.n_rb,
                     v.W, v.slot, v.slotY, C, listC, cntC, cmask, Y, actY, part);
  const size_t n = (size_t)v.G * v.W;
  hipLaunchKernelGGL(k_coldot_sum, dim3(nblk(n, 256)), dim3(256), 0, s, n, part, out);
}

// ---------------------------------------------------------------------------------------
// orthonormalization (section 3.4): scales, normalized overlaps D and eta, normalization
// of C, selection of the pairs, the combination C <- C - 1/2 C D_sel with truncation
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ bool col_in_scope(int c, int OW, int nocc, int nvirt, int occ_only) {
  if (c < OW) return c < nocc;
  if (occ_only) return false;
  return c - OW < nvirt;
}

__global__ void k_ortho_scale(int G, int W, int OW, const int* self_pair, const double* O, const int* pnocc,
                              const int* pnvirt, int occ_only, double* sc, Scalars* sd) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= G * W) return;
  const int g = idx / W, c = idx % W;
  double v = 1.0;
  if (col_in_scope(c, OW, pnocc[g], pnvirt[g], occ_only)) {
    const double d = O[(size_t)self_pair[g] * W * W + (size_t)c * W + c];
    if (!(d > 0.0)) sd->err = 1;
    else v = sqrt(d);
  }
  sc[idx] = v;
}
void launch_ortho_scale(const View& v, int, const int* self_pair, const double* O, const int* pnocc,
                        const int* pnvirt, int occ_only, double* sc, Scalars* sd, hipStream_t s) {
  const int n = v.G * v.W;
  hipLaunchKernelGGL(k_ortho_scale, dim3(nblk(n, 256)), dim3(256), 0, s, v.G, v.W, v.OW, self_pair, O, pnocc,
                     pnvirt, occ_only, sc, sd);
}

// D = normalized O with the diagonal of the self pair removed; also writes the transpose
// of each off-diagonal block (Dt[p] = D[p]^T) so that both orientations load coalesced.
__global__ void __launch_bounds__(256) k_normalize_d(int W, int OW, const int* pg, const int* ph, double* O,
                                                     double* Dt, const double* sc, const int* pnocc,
                                                     const int* pnvirt, int occ_only, Scalars* sd) {
  __shared__ double tb[16][17];
  const int p = blockIdx.x;
  const int g = pg[p], h = ph[p];
  const int nog = pnocc[g], nvg = pnvirt[g], noh = pnocc[h], nvh = pnvirt[h];
  double* Op = O + (size_t)p * W * W;
  double* Tp = Dt + (size_t)p * W * W;
  const int ii = threadIdx.x >> 4, jj = threadIdx.x & 15;
  double m = 0.0;
  for (int ti = 0; ti < W; ti += 16)
    for (int tj = 0; tj < W; tj += 16) {
      const int i = ti + ii, j = tj + jj;
      const size_t e = (size_t)i * W + j;
      double d = 0.0;
      if (col_in_scope(i, OW, nog, nvg, occ_only) && col_in_scope(j, OW, noh, nvh, occ_only) &&
          !(g == h && i == j)) {
        d = Op[e] / (sc[(size_t)g * W + i] * sc[(size_t)h * W + j]);
        m = fmax(m, fabs(d));
      }
      Op[e] = d;
      if (g != h) {
        tb[ii][jj] = d;
        __syncthreads();
        Tp[(size_t)(tj + ii) * W + ti + jj] = tb[jj][ii];
        __syncthreads();
      }
    }
  block_max_to(m, &sd->eta_bits);
}
void launch_normalize_d(const View& v, int n_pairs, const int* pg, const int* ph, double* O, double* Dt,
                        const double* sc, const int* pnocc, const int* pnvirt, int occ_only, Scalars* sd,
                        hipStream_t s) {
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_normalize_d, dim3(n_pairs), dim3(256), 0, s, v.W, v.OW, pg, ph, O, Dt, sc, pnocc, pnvirt,
                       occ_only, sd);
}

// Workgroups per group of the kernels that stride over a group's listed tiles (the lists are
// on the device, so the grid cannot be sized by their lengths)
constexpr int TILE_STRIDE_WG = 64;

__global__ void __launch_bounds__(256) k_scale_c(int n_rb, int W, const int* slot, double* C, const int* listC,
                                                 const int* cntC, const unsigned int* cmask, const double* sc) {
  __shared__ int s_so[256];
  __shared__ unsigned int s_cm[256];
  const int g = blockIdx.y;
  const double* s = sc + (size_t)g * W;
  const size_t gb = (size_t)g * n_rb;
  const int cnt = cntC[g];
  const int mine = cnt > (int)blockIdx.x ? (cnt - (int)blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
  for (int i0 = 0; i0 < mine; i0 += 256) {
    // the slots and slice masks of 256 of this workgroup's tiles, one per thread
    {
      const int i = i0 + (int)threadIdx.x;
      int so = 0;
      unsigned int cm = 0u;
      if (i < mine) {
        const size_t tile = gb + listC[gb + blockIdx.x + (size_t)gridDim.x * i];
        so = slot[tile];
        cm = cmask[tile];
      }
      s_so[threadIdx.x] = so;
      s_cm[threadIdx.x] = cm;
    }
    __syncthreads();
    const int nb = mine - i0 < 256 ? mine - i0 : 256;
    for (int j = 0; j < nb; ++j) {
      double* Ct = C + (size_t)s_so[j] * (RB * W);
      const unsigned int cm = s_cm[j];
      for (int e = threadIdx.x; e < RB * W; e += 256) {
        const int c = e % W;
        if ((cm >> (c >> 4)) & 1u) Ct[e] = Ct[e] / s[c];     // a zero slice stays zero
      }
    }
    __syncthreads();
  }
}
void launch_scale_c(const View& v, double* C, const int* listC, const int* cntC, const unsigned int* cmask,
                    const double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_c, dim3(std::min(v.n_rb, TILE_STRIDE_WG), v.G), dim3(256), 0, s, v.n_rb, v.W, v.slot, C,
                     listC, cntC, cmask, sc);
}

// Per pair: flag it when any |D| >= 1e-3 eta, flag the MOs that take part, and record for
// every row of D (orientation 0: rows = MOs of pg[p], rmask[(2p) W + i]) and of its transpose
// (orientation 1: rows = MOs of ph[p], rmask[(2p + 1) W + j]) the 16-column slices of the other
// group that hold a selected entry (bit n = slice n).  nsel (work counting, may be NULL): the
// selected ordered pairs (i, j), i != j, per MO i, added over the pairs.
__global__ void __launch_bounds__(256) k_mark_selected(int W, const int* pg, const int* ph, const double* D,
                                                       const Scalars* sd, uint8_t* pair_sel, uint8_t* upd,
                                                       uint8_t* rmask, int* nsel) {
  const int p = blockIdx.x;
  const int g = pg[p], h = ph[p];
  __shared__ unsigned int r0[MAX_W], r1[MAX_W];
  __shared__ int n0[MAX_W], n1[MAX_W];
  for (int c = threadIdx.x; c < MAX_W; c += 256) { r0[c] = 0u; r1[c] = 0u; n0[c] = 0; n1[c] = 0; }
  __syncthreads();
  const double thr = 1e-3 * __longlong_as_double((long long)sd->eta_bits);
  const double* Dp = D + (size_t)p * W * W;
  int any = 0;
  for (int e = threadIdx.x; e < W * W; e += 256) {
    if (fabs(Dp[e]) >= thr && Dp[e] != 0.0) {
      const int i = e / W, j = e % W;
      any = 1;
      upd[(size_t)g * W + i] = 1;
      upd[(size_t)h * W + j] = 1;
      atomicOr(&r0[i], 1u << (j >> 4));
      atomicOr(&r1[j], 1u << (i >> 4));
      if (nsel) { atomicAdd(&n0[i], 1); atomicAdd(&n1[j], 1); }
    }
  }
  any = __syncthreads_or(any);
  uint8_t* rm = rmask + (size_t)p * 2 * W;
  for (int c = threadIdx.x; c < W; c += 256) {
    rm[c] = (uint8_t)r0[c];
    rm[W + c] = (uint8_t)r1[c];
    if (nsel) {
      // a self pair holds both (i, j) and (j, i); another pair only (i, j) with i of g
      if (n0[c]) atomicAdd(&nsel[(size_t)g * W + c], n0[c]);
      if (g != h && n1[c]) atomicAdd(&nsel[(size_t)h * W + c], n1[c]);
    }
  }
  if (threadIdx.x == 0) pair_sel[p] = (uint8_t)(any ? 1 : 0);
}
void launch_mark_selected(const View& v, int n_pairs, const int* pg, const int* ph, const double* D,
                          const Scalars* sd, uint8_t* pair_sel, uint8_t* upd, uint8_t* rmask, int* nsel,
                          hipStream_t s) {
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_mark_selected, dim3(n_pairs), dim3(256), 0, s, v.W, pg, ph, D, sd, pair_sel, upd, rmask,
                       nsel);
}

// Output tiles of the combination: act_new[g][r] is set where C_g is active at r or where a
// neighbour h with a selected pair is.  Scattered from the lists of active tiles (act_new is
// cleared first): one wave per item, an item being a selected pair in one orientation (target
// group, source group) or a group's own tiles; the lanes walk the source's list.  Without a
// mask, a target tile with no slot gets 2: the combination there is computed and must come
// out zero (its values are the neighbours' tails times D_sel, mostly below the cut).  With a
// mask, only masked tiles are set (to 1).  Every write to a tile stores the same value.
__global__ void __launch_bounds__(256) k_update_support(int G, int n_rb, int n_pairs, const int* __restrict__ slot,
                                                        const int* __restrict__ listC, const int* __restrict__ cntC,
                                                        const int* __restrict__ pg, const int* __restrict__ ph,
                                                        const uint8_t* __restrict__ pair_sel,
                                                        const uint8_t* __restrict__ mask,
                                                        uint8_t* __restrict__ act_new) {
  const int item = (int)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int tgt, src;
  if (item < 2 * n_pairs) {
    const int p = item >> 1;
    if (!pair_sel[p]) return;
    tgt = (item & 1) ? ph[p] : pg[p];
    src = (item & 1) ? pg[p] : ph[p];
    if ((item & 1) && tgt == src) return;      // a group's pair with itself, once
  } else if (item < 2 * n_pairs + G) {
    tgt = src = item - 2 * n_pairs;
  } else {
    return;
  }
  const int lane = threadIdx.x & 63;
  const size_t sb = (size_t)src * n_rb, tb = (size_t)tgt * n_rb;
  const int n_t = cntC[src];
  for (int t = lane; t < n_t; t += 64) {
    const size_t idx = tb + listC[sb + t];
    if (mask) {
      if (mask[idx]) act_new[idx] = 1;
    } else {
      act_new[idx] = slot[idx] < 0 ? 2 : 1;
    }
  }
}
void launch_update_support(const View& v, const int* listC, const int* cntC, int n_pairs, const int* pg,
                           const int* ph, const uint8_t* pair_sel, const uint8_t* mask, uint8_t* act_new,
                           hipStream_t s) {
  launch_fill_u8(act_new, (size_t)v.G * v.n_rb, 0, s);
  const int items = 2 * n_pairs + v.G;
  hipLaunchKernelGGL(k_update_support, dim3((items + 3) / 4), dim3(256), 0, s, v.G, v.n_rb, n_pairs, v.slot, listC,
                     cntC, pg, ph, pair_sel, mask, act_new);
}

// activity flags and slice masks of the listed tiles back to zero (the values are not touched)
__global__ void __launch_bounds__(256) k_clear_flags(int n_rb, uint8_t* act, unsigned int* cmask, const int* list,
                                                     const int* cnt) {
  const int g = blockIdx.y;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= cnt[g]) return;
  const size_t tile = (size_t)g * n_rb + list[(size_t)g * n_rb + t];
  act[tile] = 0;
  cmask[tile] = 0u;
}
void launch_clear_flags(const View& v, uint8_t* act, unsigned int* cmask, const int* list, const int* cnt,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_clear_flags, dim3((v.n_rb + 255) / 256, v.G), dim3(256), 0, s, v.n_rb, act, cmask, list, cnt);
}

// ---------------------------------------------------------------------------------------
// Column scans of C tiles (one wave per listed tile; lane l owns columns l and l + 64).
//  * k_tile_flags: the activity byte, the 16-column slice mask and (colm, may be NULL) the
//    nonzero columns of each tile, exactly from its values.
//  * k_pack_cols: the nonzero columns of each tile packed to the front of its slot in P (a
//    buffer of the pool of Y, addressed with slotY, whose tiles include all of C's),
//    column-major (packed column k = the 16 rows of the tile's k-th nonzero column, one
//    128-byte line), with cidx[tile W + k] its column and ncol[tile] their number.  Only
//    columns below col_end are packed (the occupied ones in an occupied-only sweep).
// ---------------------------------------------------------------------------------------

template <int NT>
__device__ __forceinline__ void tile_columns(const double* __restrict__ T, int col_end, double (&v0)[RB],
                                             double (&v1)[RB], bool& nz0, bool& nz1) {
  constexpr int W = NT * 16;
  const int lane = threadIdx.x & 63;
  const bool in0 = lane < W && lane < col_end, in1 = lane + 64 < W && lane + 64 < col_end;
  nz0 = nz1 = false;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    v0[k] = in0 ? T[k * W + lane] : 0.0;
    nz0 |= v0[k] != 0.0;
    if constexpr (W > 64) {
      v1[k] = in1 ? T[k * W + lane + 64] : 0.0;
      nz1 |= v1[k] != 0.0;
    } else {
      v1[k] = 0.0;
    }
  }
}

template <int NT>
__global__ void __launch_bounds__(256) k_tile_flags(int G, int n_rb, int nchunk, const int* __restrict__ slot,
                                                    const double* __restrict__ C,
                                                    const int* __restrict__ list, const int* __restrict__ cnt,
                                                    uint8_t* __restrict__ act, unsigned int* __restrict__ cmask,
                                                    ulonglong2* __restrict__ colm) {
  constexpr int W = NT * 16;
  int chunk;
  const int g = xcd_group_chunk(nchunk, chunk);
  if (g >= G) return;
  const int n_t = cnt[g];
  for (int t = chunk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); t < n_t; t += 4 * nchunk) {
    const size_t tile = (size_t)g * n_rb + list[(size_t)g * n_rb + t];
    double v0[RB], v1[RB];
    bool nz0, nz1;
    tile_columns<NT>(C + (size_t)slot[tile] * (RB * W), W, v0, v1, nz0, nz1);
    const unsigned long long b0 = __ballot(nz0), b1 = __ballot(nz1);
    unsigned int cm = 0u;
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const unsigned long long b = n < 4 ? b0 : b1;
      if ((b >> (16 * (n & 3))) & 0xffffull) cm |= 1u << n;
    }
    if ((threadIdx.x & 63) == 0) {
      cmask[tile] = cm;
      act[tile] = (uint8_t)(cm != 0u);
      if (colm) colm[tile] = make_ulonglong2(b0, b1);
    }
  }
}

template <int NT>
__global__ void __launch_bounds__(256) k_pack_cols(int G, int n_rb, int nchunk, const int* __restrict__ slot,
                                                   const int* __restrict__ slotP, const double* __restrict__ C,
                                                   const int* __restrict__ list, const int* __restrict__ cnt,
                                                   int col_end, const double* __restrict__ sc,
                                                   double* __restrict__ P, uint8_t* __restrict__ cidx,
                                                   uint8_t* __restrict__ ncol) {
  constexpr int W = NT * 16;
  int chunk;
  const int g = xcd_group_chunk(nchunk, chunk);
  if (g >= G) return;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  // the columns' norms of the sweep (1 for a column out of its scope): P holds C's columns
  // divided by them, as k_scale_c would have left them
  const double s0 = lane < W ? sc[(size_t)g * W + lane] : 1.0;
  const double s1 = lane + 64 < W ? sc[(size_t)g * W + lane + 64] : 1.0;
  const int n_t = cnt[g];
  for (int t = chunk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); t < n_t; t += 4 * nchunk) {
    const size_t tile = (size_t)g * n_rb + list[(size_t)g * n_rb + t];
    double v0[RB], v1[RB];
    bool nz0, nz1;
    tile_columns<NT>(C + (size_t)slot[tile] * (RB * W), col_end, v0, v1, nz0, nz1);
    const unsigned long long b0 = __ballot(nz0), b1 = __ballot(nz1);
    const int c0 = __popcll(b0);
    const size_t sp = (size_t)slotP[tile];
    double* Pt = P + sp * (RB * W);
    uint8_t* ct = cidx + sp * W;
    if (nz0) {
      const int k = __popcll(b0 & below);
#pragma unroll
      for (int r = 0; r < RB; ++r) Pt[k * RB + r] = v0[r] / s0;
      ct[k] = (uint8_t)lane;
    }
    if (nz1) {
      const int k = c0 + __popcll(b1 & below);
#pragma unroll
      for (int r = 0; r < RB; ++r) Pt[k * RB + r] = v1[r] / s1;
      ct[k] = (uint8_t)(lane + 64);
    }
    if (lane == 0) ncol[tile] = (uint8_t)(c0 + __popcll(b1));
  }
}

void launch_tile_flags(const View& v, const double* C, const int* list, const int* cnt, uint8_t* act,
                       unsigned int* cmask, ulonglong2* colm, hipStream_t s) {
  const int nchunk = tile_list_chunks(v.G, v.max_c);
  dim3 grid(xcd_grid(v.G, nchunk)), blk(256);
  switch (v.W / 16) {
#define SSCF_TF(NT) case NT: hipLaunchKernelGGL(k_tile_flags<NT>, grid, blk, 0, s, v.G, v.n_rb, nchunk, v.slot, C, list, cnt, act, cmask, colm); break;
    SSCF_TF(1) SSCF_TF(2) SSCF_TF(3) SSCF_TF(4) SSCF_TF(5) SSCF_TF(6) SSCF_TF(7) SSCF_TF(8)
#undef SSCF_TF
  }
}

void launch_pack_cols(const View& v, const double* C, const int* list, const int* cnt, int col_end,
                      const double* sc, double* P, uint8_t* cidx, uint8_t* ncol, hipStream_t s) {
  const int nchunk = tile_list_chunks(v.G, v.max_c);
  dim3 grid(xcd_grid(v.G, nchunk)), blk(256);
  switch (v.W / 16) {
#define SSCF_PK(NT) case NT: hipLaunchKernelGGL(k_pack_cols<NT>, grid, blk, 0, s, v.G, v.n_rb, nchunk, v.slot, v.slotY, C, list, cnt, col_end, sc, P, cidx, ncol); break;
    SSCF_PK(1) SSCF_PK(2) SSCF_PK(3) SSCF_PK(4) SSCF_PK(5) SSCF_PK(6) SSCF_PK(7) SSCF_PK(8)
#undef SSCF_PK
  }
}

// Cn[g][r] = C[g][r] - 1/2 sum_{h ~ g} C[h][r] D_sel(h, g), then |v| < cut -> 0 in the
// columns that took part in a combination.  C enters divided by the sweep's column norms sc
// (the normalization of section 3.4, applied here and in the packing rather than in a pass of
// its own; the last sweep of a loop, which combines nothing, runs k_scale_c instead).  D is stored per unordered pair (a <= b) with
// rows = MOs of a, columns = MOs of b; Dt holds the transposes, so D_sel(h, g) (rows = MOs
// of h) is read row-contiguously in both orientations.
//
// Cn may be C itself (the update runs in place): the wave of tile (g, r) is the only one that
// reads or writes C's tile (g, r); the other groups' tiles come from their packed copy.
// One wave per output tile (g, r) at a time, walking g's list of output tiles (see
// tile_list_chunks), with no workgroup synchronization.  A ballot over g's
// neighbours finds, 64 at a time, those h whose pair is selected and whose tile (h, r) has a
// nonzero column.  Per such h only the tile's nonzero columns enter the product: they come
// packed (k_pack_cols), four per k-step of the 16 x 16 x 4 matrix-core product, each as one
// 128-byte line; the B operand is the matching rows of D_sel(h, g) (thresholded at 1e-3
// eta), and a 16-column slice of the output is skipped for a k-step when none of its four
// rows holds a selected entry there (rmask).  Adding the skipped terms would add exact
// zeros.  The sum runs over h in neighbour order and over the packed columns in increasing
// column order, so the result does not depend on the launch.  Four waves per SIMD are asked
// for: the walk over the list would otherwise keep more registers live and leave three.
template <int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_ortho_update(int G, int n_rb, int nchunk, const int* __restrict__ slot,
               const int* __restrict__ slotP, const double* C,
               const uint8_t* __restrict__ actC, const unsigned int* __restrict__ cmaskC,
               const double* __restrict__ P, const uint8_t* __restrict__ cidx,
               const uint8_t* __restrict__ ncol,
               const int* __restrict__ gn_ptr, const int* __restrict__ gn,
               const int* __restrict__ pair_of,
               const uint8_t* __restrict__ pair_sel,
               const double* __restrict__ D, const double* __restrict__ Dt,
               const uint8_t* __restrict__ rmask,
               const Scalars* __restrict__ sd,
               const uint8_t* __restrict__ upd, const double* __restrict__ sc, double cut,
               const int* __restrict__ listN, const int* __restrict__ cntN,
               double* Cn, uint8_t* __restrict__ actN,
               unsigned int* __restrict__ cmaskN, int* __restrict__ cap_err,
               unsigned long long* ctr) {
  constexpr int W = NT * 16;
  constexpr int KB = 2;                       // k-steps whose loads go out together
  int chunk;
  const int g = xcd_group_chunk(nchunk, chunk);
  if (g >= G) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const double thr = 1e-3 * __longlong_as_double((long long)sd->eta_bits);
  const int k_end = gn_ptr[g + 1];
  const int n_t = cntN[g];
  for (int t = chunk * 4 + wv; t < n_t; t += 4 * nchunk) {
    const int r = listN[(size_t)g * n_rb + t];
    d4 acc[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[n] = d4{0.0, 0.0, 0.0, 0.0};
    unsigned int n_mfma = 0;
    for (int kb = gn_ptr[g]; kb < k_end; kb += 64) {
      const int k = kb + lane;
      int h = 0, nz = 0, pk = 0, shk = 0;
      if (k < k_end) {
        h = gn[k];
        const size_t th = (size_t)h * n_rb + r;
        pk = pair_of[(size_t)g * G + h];
        if (pair_sel[pk] && actC[th]) {
          nz = ncol[th];
          shk = slotP[th];                     // every lane's pair and slot in one round trip
        }
      }
      unsigned long long M = __ballot(nz != 0);
      // the next neighbour's packed column indices load while the current one multiplies
      int jn = -1, col0n = 0, col1n = 0;
      auto fetch_cols = [&]() {
        jn = __ffsll((long long)M) - 1;
        M &= M - 1ull;
        const int nzn = __builtin_amdgcn_readfirstlane(__shfl(nz, jn));
        const size_t shn = (size_t)(unsigned int)__builtin_amdgcn_readfirstlane(__shfl(shk, jn));
        const uint8_t* ci = cidx + shn * W;      // packed column k's index lives in lane k or k - 64
        col0n = lane < nzn ? ci[lane] : 0;
        col1n = (W > 64 && lane + 64 < nzn) ? ci[lane + 64] : 0;
      };
      if (M) fetch_cols();
      while (jn >= 0) {
        const int j = jn;
        const int col0 = col0n, col1 = col1n;
        const int hc = __builtin_amdgcn_readfirstlane(__shfl(h, j));
        const int nzj = __builtin_amdgcn_readfirstlane(__shfl(nz, j));
        const int p = __builtin_amdgcn_readfirstlane(__shfl(pk, j));
        const bool tr = hc > g;
        const double* Dp = (tr ? Dt : D) + (size_t)p * W * W + lr;
        const uint8_t* rm = rmask + ((size_t)p * 2 + (tr ? 1 : 0)) * W;
        const size_t sh = (size_t)(unsigned int)__builtin_amdgcn_readfirstlane(__shfl(shk, j));
        const double* A = P + sh * (RB * W) + lr;
        int m0 = lane < nzj ? rm[col0] : 0;
        int m1 = (W > 64 && lane + 64 < nzj) ? rm[col1] : 0;
        jn = -1;
        if (M) fetch_cols();
        // OR over the four columns of each k-step (aligned groups of four lanes)
        m0 |= __shfl_xor(m0, 1);
        m0 |= __shfl_xor(m0, 2);
        m1 |= __shfl_xor(m1, 1);
        m1 |= __shfl_xor(m1, 2);
        for (int s0 = 0; s0 < nzj; s0 += 4 * KB) {
          double a[KB];
          int col[KB];
          unsigned int nm[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) {
            const int q0 = s0 + 4 * u;           // first packed column of this k-step
            const int kk = q0 + lk;
            a[u] = kk < nzj ? A[kk * RB] : 0.0;
            const int c0 = __shfl(col0, kk & 63), c1 = __shfl(col1, kk & 63);
            col[u] = q0 < 64 ? c0 : c1;
            unsigned int mm = 0u;
            if (q0 < nzj) mm = (unsigned int)(q0 < 64 ? __builtin_amdgcn_readlane(m0, q0 & 63)
                                                       : __builtin_amdgcn_readlane(m1, q0 & 63));
            nm[u] = mm;
          }
          double b[KB][NT];
#pragma unroll
          for (int u = 0; u < KB; ++u)
#pragma unroll
            for (int n = 0; n < NT; ++n) b[u][n] = ((nm[u] >> n) & 1u) ? Dp[(size_t)col[u] * W + n * 16] : 0.0;
#pragma unroll
          for (int u = 0; u < KB; ++u)
#pragma unroll
            for (int n = 0; n < NT; ++n)
              if ((nm[u] >> n) & 1u) {
                const double bv = (fabs(b[u][n]) >= thr) ? b[u][n] : 0.0;
                acc[n] = mfma64(a[u], bv, acc[n]);
                ++n_mfma;
              }
        }
      }
    }
    const size_t tile = (size_t)g * n_rb + r;
    const int so_i = slot[tile];
    if (so_i < 0) {
      // a tile with no slot (listed with activity 2): C is zero there; the combination must
      // leave it so after the cut, else C has outgrown its capacity
      int bad = 0;
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const bool u = upd[(size_t)g * W + n * 16 + lr] != 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double v = -0.5 * acc[n][q];
          bad |= (u ? fabs(v) >= cut : v != 0.0);
        }
      }
      if (__ballot(bad) && lane == 0) note_capacity(cap_err, tile);
      if (lane == 0) {
        actN[tile] = 0;
        cmaskN[tile] = 0u;
        if (ctr && n_mfma) atomicAdd(ctr, (unsigned long long)n_mfma);
      }
      continue;
    }
    // a 16-column slice whose flag is clear holds zeros (C's pool starts zeroed, and every
    // writer of C leaves the flags exact for the values it stores): it is not read, and it is
    // not written when the combination adds nothing to it
    const unsigned int cm_old = actC[tile] ? cmaskC[tile] : 0u;
    const size_t so = (size_t)so_i;
    const double* Cg = C + so * (RB * W);
    double* Co = Cn + so * (RB * W);
    unsigned int cm = 0;
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int jj = n * 16 + lr;
      const bool u = upd[(size_t)g * W + jj] != 0;
      const bool was = (cm_old >> n) & 1u;
      const double sg = was ? sc[(size_t)g * W + jj] : 1.0;
      const bool hit = __ballot(acc[n][0] != 0.0 || acc[n][1] != 0.0 || acc[n][2] != 0.0 || acc[n][3] != 0.0) != 0ull;
      const bool put = was || hit;
      int nz = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lk + 4 * q;
        double v = (was ? Cg[i * W + jj] / sg : 0.0) - 0.5 * acc[n][q];
        if (u && fabs(v) < cut) v = 0.0;
        if (put) Co[i * W + jj] = v;
        nz |= (v != 0.0);
      }
      if (__ballot(nz)) cm |= 1u << n;
    }
    if (lane == 0) {
      actN[tile] = (uint8_t)(cm != 0u);
      cmaskN[tile] = cm;
      if (ctr && n_mfma) atomicAdd(ctr, (unsigned long long)n_mfma);
    }
  }
}

void launch_ortho_update(const View& v, const double* C, const uint8_t* actC, const unsigned int* cmaskC,
                         const double* P, const uint8_t* cidx,
                         const uint8_t* ncol, const int* gn_ptr, const int* gn, const int* pair_of,
                         const uint8_t* pair_sel, const double* D, const double* Dt, const uint8_t* rmask,
                         const Scalars* sd, const uint8_t* upd, const double* sc, double cut, const int* listN,
                         const int* cntN,
                         double* Cn, uint8_t* actN, unsigned int* cmaskN, unsigned long long* ctr, hipStream_t s) {
  const int nchunk = tile_list_chunks(v.G, v.n_rb);
  dim3 grid(xcd_grid(v.G, nchunk)), blk(256);
  switch (v.W / 16) {
#define SSCF_UPD(NT) case NT: hipLaunchKernelGGL(k_ortho_update<NT>, grid, blk, 0, s, v.G, v.n_rb, nchunk, v.slot, v.slotY, C, actC, cmaskC, P, cidx, ncol, gn_ptr, gn, pair_of, pair_sel, D, Dt, rmask, sd, upd, sc, cut, listN, cntN, Cn, actN, cmaskN, v.cap_err, ctr); break;
    SSCF_UPD(1) SSCF_UPD(2) SSCF_UPD(3) SSCF_UPD(4) SSCF_UPD(5) SSCF_UPD(6) SSCF_UPD(7) SSCF_UPD(8)
#undef SSCF_UPD
  }
}

// ---------------------------------------------------------------------------------------
// DFTB Fock matrix (section 3.7): Q = gamma dq over all atom pairs, unscreened, then
// H = H0 + 1/2 S (Q_a + Q_b) with |H| < eps -> 0 (section 4.1)
// ---------------------------------------------------------------------------------------

// Atom a's sum over b is split into CL_SPLIT contiguous ranges of b, one workgroup each
// (the grid then fills the chip); k_coulomb_sum adds the ranges' sums in a fixed order.

__global__ void __launch_bounds__(256) k_coulomb(int n, int scc, const double* __restrict__ xyz,
                                                 const double* __restrict__ U, const double* __restrict__ dq,
                                                 double* __restrict__ part) {
  __shared__ double sx[256], sy[256], sz[256], siu[256], sq[256];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = a < n;
  const double xa = live ? xyz[3 * a] : 0.0, ya = live ? xyz[3 * a + 1] : 0.0, za = live ? xyz[3 * a + 2] : 0.0;
  const double ua = live ? U[a] : 0.0, ia = live ? 1.0 / ua : 0.0;
  const int per = (n + CL_SPLIT - 1) / CL_SPLIT;
  const int b0 = blockIdx.y * per, b1 = min(n, b0 + per);
  double s = 0.0;
  for (int base = b0; base < b1; base += 256) {
    const int x = base + threadIdx.x;
    __syncthreads();
    if (x < b1) {
      sx[threadIdx.x] = xyz[3 * x]; sy[threadIdx.x] = xyz[3 * x + 1]; sz[threadIdx.x] = xyz[3 * x + 2];
      siu[threadIdx.x] = 1.0 / U[x]; sq[threadIdx.x] = dq[x];
    }
    __syncthreads();
    const int m = min(256, b1 - base);
    if (live && scc) {
      for (int k = 0; k < m; ++k) {
        double gam;
        if (base + k == a) {
          gam = ua;
        } else {
          const double dx = xa - sx[k], dy = ya - sy[k], dz = za - sz[k];
          const double u = 0.5 * (ia + siu[k]);
          gam = 1.0 / sqrt(dx * dx + dy * dy + dz * dz + u * u);
        }
        s += gam * sq[k];
      }
    }
  }
  if (live) part[(size_t)blockIdx.y * n + a] = s;
}
__global__ void k_coulomb_sum(int n, const double* part, double* Q) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double s = 0.0;
  for (int sp = 0; sp < CL_SPLIT; ++sp) s += part[(size_t)sp * n + a];
  Q[a] = s;
}
void launch_coulomb(const View& v, int scc, const double* dq, double* part, double* Q, hipStream_t s) {
  hipLaunchKernelGGL(k_coulomb, dim3(nblk(v.n_atoms, 256), CL_SPLIT), dim3(256), 0, s, v.n_atoms, scc, v.xyz, v.U,
                     dq, part);
  hipLaunchKernelGGL(k_coulomb_sum, dim3(nblk(v.n_atoms, 256)), dim3(256), 0, s, v.n_atoms, part, Q);
}

__global__ void k_fock(size_t n, int n_ao, const int* xs_row, const int* xs_col, const int* ao_atom,
                       const double* S, const double* H0, const double* Hfull, const double* Q, double eps,
                       double* H, float* H32) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const size_t b = e >> 8;
  const int i = (int)((e >> 4) & 15), j = (int)(e & 15);
  const int mu = xs_row[b] * RB + i, nu = xs_col[b] * RB + j;
  double h = 0.0;
  if (mu < n_ao && nu < n_ao) {
    if (Hfull) h = Hfull[e];
    else h = H0[e] + 0.5 * S[e] * (Q[ao_atom[mu]] + Q[ao_atom[nu]]);
  }
  h = (fabs(h) < eps) ? 0.0 : h;
  H[e] = h;
  if (H32) H32[e] = (float)h;
}
void launch_fock(const View& v, const double* S, const double* H0, const double* Hfull, const double* Q, double eps,
                 double* H, float* H32, hipStream_t s) {
  const size_t n = (size_t)v.nbx * 256;
  hipLaunchKernelGGL(k_fock, dim3(nblk(n, 256)), dim3(256), 0, s, n, v.n_ao, v.xs_row, v.xs_col, v.ao_atom, S, H0,
                     Hfull, Q, eps, H, H32);
}

// ---------------------------------------------------------------------------------------
// rotation selection (section 3.5): candidates |F_ia| >= eps (F != 0); at most K of them,
// the largest |F| first with ties by (i, a); inside each Jacobi block ordered by
// decreasing |F| then (i, a); angle from the F of the start of the step
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ bool cand_of(const double* F, size_t e, int OW, int VW, const int* jb_nocc,
                                        const int* jb_nvirt, double tau, double& f, int& b, int& i, int& a,
                                        bool& valid) {
  const size_t per = (size_t)OW * VW;
  b = (int)(e / per);
  const int rem = (int)(e % per);
  i = rem / VW;
  a = rem % VW;
  valid = i < jb_nocc[b] && a < jb_nvirt[b];
  f = F[e];
  return valid && f != 0.0 && fabs(f) >= tau;
}

__global__ void __launch_bounds__(256) k_count_candidates(size_t n, int OW, int VW, const int* jb_nocc,
                                                          const int* jb_nvirt, const double* F, double tau,
                                                          Scalars* sd) {
  __shared__ int cs[4];
  int c = 0;
  double m = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double f; int b, i, a; bool valid;
    if (cand_of(F, e, OW, VW, jb_nocc, jb_nvirt, tau, f, b, i, a, valid)) ++c;
    if (valid) m = fmax(m, fabs(f));
  }
  c = wave_sum_i(c);
  if ((threadIdx.x & 63) == 0) cs[threadIdx.x >> 6] = c;
  block_max_to(m, &sd->fov_bits);
  if (threadIdx.x == 0) atomicAdd(&sd->n_cand, cs[0] + cs[1] + cs[2] + cs[3]);
}
void launch_count_candidates(int nb, int OW, int VW, const int* jb_nocc, const int* jb_nvirt, const double* F,
                             double tau, Scalars* sd, hipStream_t s) {
  const size_t n = (size_t)nb * OW * VW;
  unsigned int g = nblk(n, 256);
  if (g > 4096) g = 4096;
  if (n) hipLaunchKernelGGL(k_count_candidates, dim3(g), dim3(256), 0, s, n, OW, VW, jb_nocc, jb_nvirt, F, tau, sd);
}

__global__ void __launch_bounds__(256) k_radix_hist(size_t n, int OW, int VW, const int* jb_nocc, const int* jb_nvirt,
                                                    const double* F, double tau, int shift, const Scalars* sd,
                                                    unsigned int* hist) {
  __shared__ unsigned int lh[256];
  lh[threadIdx.x] = 0;
  __syncthreads();
  const unsigned long long prefix = sd->prefix, mask = sd->mask;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double f; int b, i, a; bool valid;
    if (!cand_of(F, e, OW, VW, jb_nocc, jb_nvirt, tau, f, b, i, a, valid)) continue;
    const unsigned long long key = dbits(fabs(f));
    if ((key & mask) != prefix) continue;
    atomicAdd(&lh[(key >> shift) & 0xFF], 1u);
  }
  __syncthreads();
  if (lh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
}

// walk the histogram from the largest digit down and fix the digit of the K-th key
__global__ void k_radix_pick(int shift, Scalars* sd, unsigned int* hist) {
  if (threadIdx.x != 0) return;
  long long acc = 0;
  for (int bin = 255; bin >= 0; --bin) {
    const long long c = hist[bin];
    if (acc + c >= sd->remaining) {
      sd->prefix |= ((unsigned long long)bin) << shift;
      sd->mask |= 0xFFULL << shift;
      sd->remaining -= acc;
      sd->tie_count = (int)c;
      break;
    }
    acc += c;
  }
  for (int bin = 0; bin < 256; ++bin) hist[bin] = 0;
}

void launch_radix_pass(int nb, int OW, int VW, const int* jb_nocc, const int* jb_nvirt, const double* F, double tau,
                       int shift, Scalars* sd, unsigned int* hist, hipStream_t s) {
  const size_t n = (size_t)nb * OW * VW;
  unsigned int g = nblk(n, 256);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_radix_hist, dim3(g), dim3(256), 0, s, n, OW, VW, jb_nocc, jb_nvirt, F, tau, shift, sd, hist);
  hipLaunchKernelGGL(k_radix_pick, dim3(1), dim3(64), 0, s, shift, sd, hist);
}

__global__ void k_sel_init(Scalars* sd, long long K, int select_all) {
  sd->prefix = 0ULL;
  sd->mask = 0ULL;
  sd->remaining = K;
  sd->cut_key = 0ULL;                 // select_all: every candidate has a key > 0
  sd->tie_cut = 0x7fffffffffffffffLL;
  sd->tie_count = 0;
  sd->tie_n = 0;
  sd->n_rot = 0;
  (void)select_all;
}
void launch_sel_init(Scalars* sd, long long K, int select_all, hipStream_t s) {
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1), 0, s, sd, K, select_all);
}

// after the radix passes: keys > prefix are all taken; `remaining` of the keys == prefix
// are needed.  cut_key is the smallest key taken.  With select-all the cut stays at 0.
__global__ void k_sel_finish(Scalars* sd) {
  sd->cut_key = sd->prefix;
  // keys == cut_key are all taken when no more of them exist than needed
  if (sd->tie_count <= sd->remaining) sd->tie_cut = 0x7fffffffffffffffLL;
  else sd->tie_cut = -1;              // resolved by launch_tie_cut
}
void launch_sel_finish(Scalars* sd, hipStream_t s) { hipLaunchKernelGGL(k_sel_finish, dim3(1), dim3(1), 0, s, sd); }

// candidates with |F| == cut_key: collect their (i * n_mo + a) keys, sort them and keep
// the `remaining` smallest (ties are taken by increasing (i, a))
__global__ void k_tie_collect(size_t n, int OW, int VW, const int* jb_g, const int* jb_h, const int* jb_nocc,
                              const int* jb_nvirt, const double* F, const int* mo_of, int W, long long n_mo,
                              double tau, Scalars* sd, long long* ties) {
  if (sd->tie_cut != -1) return;
  const unsigned long long cut = sd->cut_key;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double f; int b, i, a; bool valid;
    if (!cand_of(F, e, OW, VW, jb_nocc, jb_nvirt, tau, f, b, i, a, valid)) continue;
    if (dbits(fabs(f)) != cut) continue;
    const long long ig = mo_of[(size_t)jb_g[b] * W + i], ag = mo_of[(size_t)jb_h[b] * W + OW + a];
    const int pos = atomicAdd(&sd->tie_n, 1);
    if (pos < MAX_TIES) ties[pos] = ig * n_mo + ag;
  }
}

__global__ void __launch_bounds__(256) k_tie_sort(Scalars* sd, const long long* ties) {
  if (sd->tie_cut != -1) return;
  __shared__ long long k[MAX_TIES];
  const int n = sd->tie_n;
  if (n > MAX_TIES) {
    if (threadIdx.x == 0) { sd->err |= 2; sd->tie_cut = 0x7fffffffffffffffLL; }
    return;
  }
  int N = 1;
  while (N < n) N <<= 1;
  for (int i = threadIdx.x; i < N; i += 256) k[i] = (i < n) ? ties[i] : 0x7fffffffffffffffLL;
  __syncthreads();
  for (int len = 2; len <= N; len <<= 1)
    for (int j = len >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += 256) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & len) == 0;
          const long long x = k[i], y = k[ixj];
          if ((x > y) == up) { k[i] = y; k[ixj] = x; }
        }
      }
      __syncthreads();
    }
  if (threadIdx.x == 0) sd->tie_cut = k[sd->remaining - 1];
}

void launch_tie_cut(int nb, int OW, int VW, const int* jb_g, const int* jb_h, const int* jb_nocc, const int* jb_nvirt,
                    const double* F, const int* mo_of, int W, long long n_mo, double tau, Scalars* sd,
                    long long* ties, hipStream_t s) {
  const size_t n = (size_t)nb * OW * VW;
  unsigned int g = nblk(n, 256);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_tie_collect, dim3(g), dim3(256), 0, s, n, OW, VW, jb_g, jb_h, jb_nocc, jb_nvirt, F, mo_of, W,
                     n_mo, tau, sd, ties);
  hipLaunchKernelGGL(k_tie_sort, dim3(1), dim3(256), 0, s, sd, ties);
}

// One workgroup per Jacobi block: the selected candidates of the block sorted by
// (|F| descending, i, a), the angle of each pair from the stale F (section 3.5):
// p = (F_ii - F_aa) / (2 F_ia), t = 1 / (p + sgn(p) sqrt(1 + p^2)), c = (1 + t^2)^(-1/2),
// s = t c, sgn(0) = +1; and the sorted set of columns the block touches.
constexpr int SEL_MAX = 4096;

__global__ void __launch_bounds__(256) k_block_select(int W, int OW, int VW, const int* jb_g, const int* jb_h,
                                                      const int* jb_nocc, const int* jb_nvirt, const double* F,
                                                      const double* Fdiag, const int* mo_of, long long n_mo,
                                                      double tau, Scalars* sd, int* rot_cnt, int2* rot_slot,
                                                      double2* rot_cs, int* tcnt, int* tcol, ulonglong2* tmask,
                                                      int fp32) {
  __shared__ unsigned long long khi[SEL_MAX];
  __shared__ unsigned int klo[SEL_MAX];
  __shared__ int n_sel;
  __shared__ uint8_t used[MAX_W];
  __shared__ int upos[MAX_W];
  const int b = blockIdx.x;
  const int g = jb_g[b], h = jb_h[b];
  const int no = jb_nocc[b], nv = jb_nvirt[b];
  const size_t per = (size_t)OW * VW;
  const double* Fb = F + (size_t)b * per;
  const unsigned long long cut = sd->cut_key;
  const long long tie_cut = sd->tie_cut;
  if (threadIdx.x == 0) n_sel = 0;
  for (int c = threadIdx.x; c < MAX_W; c += 256) used[c] = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < (int)per; e += 256) {
    const int i = e / VW, a = e % VW;
    if (i >= no || a >= nv) continue;
    const double f = Fb[e];
    if (f == 0.0 || fabs(f) < tau) continue;
    const unsigned long long key = dbits(fabs(f));
    bool sel = key > cut;
    if (key == cut) {
      const long long ia = (long long)mo_of[(size_t)g * W + i] * n_mo + mo_of[(size_t)h * W + OW + a];
      sel = ia <= tie_cut;
    }
    if (!sel) continue;
    const int pos = atomicAdd(&n_sel, 1);
    khi[pos] = ~key;                       // ascending order = decreasing |F|
    klo[pos] = ((unsigned)i << 16) | (unsigned)a;
  }
  __syncthreads();
  const int n = n_sel;
  int N = 1;
  while (N < n) N <<= 1;
  for (int i = n + threadIdx.x; i < N; i += 256) { khi[i] = ~0ULL; klo[i] = ~0u; }
  __syncthreads();
  for (int len = 2; len <= N; len <<= 1)
    for (int j = len >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += 256) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & len) == 0;
          const unsigned long long x1 = khi[i], y1 = khi[ixj];
          const unsigned int x2 = klo[i], y2 = klo[ixj];
          const bool gt = (x1 > y1) || (x1 == y1 && x2 > y2);
          if (gt == up) { khi[i] = y1; khi[ixj] = x1; klo[i] = y2; klo[ixj] = x2; }
        }
      }
      __syncthreads();
    }
  // touched columns (ascending) and the slot of each column
  for (int q = threadIdx.x; q < n; q += 256) {
    used[klo[q] >> 16] = 1;
    used[OW + (klo[q] & 0xFFFF)] = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int u = 0;
    unsigned long long t0 = 0ull, t1 = 0ull;
    for (int c = 0; c < W; ++c)
      if (used[c]) {
        upos[c] = u;
        tcol[(size_t)b * W + u] = c;
        ++u;
        if (c < 64) t0 |= 1ull << c;
        else t1 |= 1ull << (c - 64);
      }
    tcnt[b] = u;
    tmask[b] = make_ulonglong2(t0, t1);
    rot_cnt[b] = n;
    atomicAdd(&sd->n_rot, n);
  }
  __syncthreads();
  const size_t rb0 = (size_t)b * per;
  for (int q = threadIdx.x; q < n; q += 256) {
    const int i = klo[q] >> 16, a = klo[q] & 0xFFFF;
    const double f = Fb[(size_t)i * VW + a];
    const double fii = Fdiag[(size_t)g * W + i], faa = Fdiag[(size_t)h * W + OW + a];
    double c, sn;
    if (fp32) {
      const float pf = ((float)fii - (float)faa) / (2.0f * (float)f);
      const float sgf = (pf >= 0.0f) ? 1.0f : -1.0f;
      const float tf = 1.0f / (pf + sgf * sqrtf(1.0f + pf * pf));
      const float cf = 1.0f / sqrtf(1.0f + tf * tf);
      c = cf;
      sn = tf * cf;
    } else {
      const double p = (fii - faa) / (2.0 * f);
      const double sg = (p >= 0.0) ? 1.0 : -1.0;
      const double t = 1.0 / (p + sg * sqrt(1.0 + p * p));
      c = 1.0 / sqrt(1.0 + t * t);
      sn = t * c;
    }
    rot_slot[rb0 + q] = make_int2(upos[i], upos[OW + a]);
    rot_cs[rb0 + q] = make_double2(c, sn);
  }
}

void launch_block_select(const View& v, int nb, const int* jb_g, const int* jb_h, const int* jb_nocc, const int* jb_nvirt,
                         const double* F, const double* Fdiag, const int* mo_of, double tau, Scalars* sd,
                         int* rot_cnt, int2* rot_slot, double2* rot_cs, int* tcnt, int* tcol, ulonglong2* tmask,
                         int fp32, hipStream_t s) {
  if (nb > 0)
    hipLaunchKernelGGL(k_block_select, dim3(nb), dim3(256), 0, s, v.W, v.OW, v.VW, jb_g, jb_h, jb_nocc, jb_nvirt, F,
                       Fdiag, mo_of, (long long)v.n_mo, tau, sd, rot_cnt, rot_slot, rot_cs, tcnt, tcol, tmask, fp32);
}

// ---------------------------------------------------------------------------------------
// rotation application.  The ordered rotations of a Jacobi block act on the block's
// touched columns as one orthogonal matrix: x -> x G_1 G_2 ... G_n = x R_b for every
// row x of C (rotations are column operations, rows are independent).  R_b is formed
// once per block (row k of R_b is e_k rotated in list order); then one workgroup per
// row block walks the rounds in order (a barrier between rounds, the blocks of a round
// spread over its waves) and applies each relevant R_b to the 16-row slice with the
// matrix cores, followed by the truncation |C| < eps of the block's columns.
// ---------------------------------------------------------------------------------------

template <typename Real>
__global__ void __launch_bounds__(128) k_compose_rot(int W, int per, const int* rot_cnt, const int2* rot_slot,
                                                     const double2* rot_cs, const int* tcnt, Real* R) {
  const int b = blockIdx.x;
  const int n = rot_cnt[b];
  if (n == 0) return;
  const int T = tcnt[b];
  const int T16 = (T + 15) & ~15;
  const int k = threadIdx.x;
  if (k >= T16) return;
  Real* row = R + ((size_t)b * W + k) * W;
  for (int j = 0; j < T16; ++j) row[j] = (j == k && k < T) ? Real(1) : Real(0);
  if (k >= T) return;
  const int2* sl = rot_slot + (size_t)b * per;
  const double2* cs = rot_cs + (size_t)b * per;
  for (int q = 0; q < n; ++q) {
    const int2 ia = sl[q];
    const Real c = (Real)cs[q].x, sn = (Real)cs[q].y;
    const Real xi = row[ia.x], xa = row[ia.y];
    row[ia.x] = c * xi + sn * xa;
    row[ia.y] = -sn * xi + c * xa;
  }
}
void launch_compose_rot(const View& v, int nb, const int* rot_cnt, const int2* rot_slot, const double2* rot_cs,
                        const int* tcnt, double* R, float* R32, hipStream_t s) {
  if (nb <= 0) return;
  if (R32)
    hipLaunchKernelGGL(k_compose_rot<float>, dim3(nb), dim3(128), 0, s, v.W, v.OW * v.VW, rot_cnt, rot_slot, rot_cs,
                       tcnt, R32);
  else
    hipLaunchKernelGGL(k_compose_rot<double>, dim3(nb), dim3(128), 0, s, v.W, v.OW * v.VW, rot_cnt, rot_slot, rot_cs,
                       tcnt, R);
}

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// FP32 16x16x4 result register r holds D[4 (l / 16) + r][l % 16]; FP64 holds D[l / 16 + 4 r][l % 16]
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ d4 op(double a, double b, d4 c) { return mfma64(a, b, c); }
  static __device__ __forceinline__ int row(int lk, int q) { return lk + 4 * q; }
};
template <> struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ f4 op(float a, float b, f4 c) { return mfma32(a, b, c); }
  static __device__ __forceinline__ int row(int lk, int q) { return 4 * lk + q; }
};

// The blocks that carry rotations, packed (block, g, h, touched columns) in round order,
// with the offset of each round: one 16-byte load per block in the rotation pass.
__global__ void __launch_bounds__(256) k_round_count(const int* round_ptr, const int* round_list, const int* rot_cnt,
                                                     int* rcnt) {
  const int r = blockIdx.x;
  int c = 0;
  for (int i = round_ptr[r] + threadIdx.x; i < round_ptr[r + 1]; i += 256) c += rot_cnt[round_list[i]] > 0;
  c = wave_sum_i(c);
  __shared__ int ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) rcnt[r] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ void k_round_prefix(int n_rounds, const int* rcnt, int* roff) {
  if (threadIdx.x != 0) return;
  int acc = 0;
  for (int r = 0; r < n_rounds; ++r) { roff[r] = acc; acc += rcnt[r]; }
  roff[n_rounds] = acc;
}

__global__ void __launch_bounds__(256) k_round_fill(const int* round_ptr, const int* round_list, const int* rot_cnt,
                                                    const int* jb_g, const int* jb_h, const int* tcnt, const int* roff,
                                                    int4* meta) {
  const int r = blockIdx.x;
  __shared__ int wsum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int base = roff[r];
  for (int i0 = round_ptr[r]; i0 < round_ptr[r + 1]; i0 += 256) {
    const int i = i0 + threadIdx.x;
    const int b = (i < round_ptr[r + 1]) ? round_list[i] : -1;
    const bool f = b >= 0 && rot_cnt[b] > 0;
    const unsigned long long m = __ballot(f);
    const int pre = __popcll(m & ((1ULL << lane) - 1ULL));
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int k = 0; k < w; ++k) off += wsum[k];
    if (f) meta[off + pre] = make_int4(b, jb_g[b], jb_h[b], tcnt[b]);
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    base += tot;
  }
}

void launch_round_meta(int n_rounds, const int* round_ptr, const int* round_list, const int* rot_cnt, const int* jb_g,
                       const int* jb_h, const int* tcnt, int* rcnt, int* roff, int4* meta, hipStream_t s) {
  if (n_rounds <= 0) return;
  hipLaunchKernelGGL(k_round_count, dim3(n_rounds), dim3(256), 0, s, round_ptr, round_list, rot_cnt, rcnt);
  hipLaunchKernelGGL(k_round_prefix, dim3(1), dim3(64), 0, s, n_rounds, rcnt, roff);
  hipLaunchKernelGGL(k_round_fill, dim3(n_rounds), dim3(256), 0, s, round_ptr, round_list, rot_cnt, jb_g, jb_h, tcnt,
                     roff, meta);
}

// One workgroup per row block rb walks the rounds in order (a barrier between rounds, the
// blocks of a round spread over its waves).  The nonzero columns of every tile (g, rb) are kept
// exact in LDS (cm_l, initialized from colm): a block is applied at rb only when one of its
// touched columns is nonzero there, and only those columns enter the product (the K dimension
// of x R_b packs them), so rows and columns the rotations cannot reach cost nothing.  After
// each block the written columns' bits are recomputed from the truncated values.  At the end
// the workgroup writes the exact activity, slice mask and column mask of each tile (g, rb).
template <int NTMAX, typename Real>
__global__ void __launch_bounds__(256) k_givens_rb(int G, int n_rb, int W, int OW, int n_rounds,
                                                   const int* __restrict__ roff, const int4* __restrict__ meta,
                                                   const ulonglong2* __restrict__ tmask,
                                                   const int* __restrict__ tcol,
                                                   const Real* __restrict__ R, double eps, const int* __restrict__ slot,
                                                   double* C, uint8_t* actC, unsigned int* cmask, ulonglong2* colm,
                                                   const int* __restrict__ rot_cnt, int* cap_err,
                                                   unsigned long long* wcnt) {
  typedef typename Mfma<Real>::acc_t acc_t;
  extern __shared__ int4 gv_smem[];
  int4* list_l = gv_smem;                                                   // relevant blocks of the round
  unsigned long long* cm_l = reinterpret_cast<unsigned long long*>(gv_smem + 256);   // 2 words per group
  uint8_t* pos_all = reinterpret_cast<uint8_t*>(cm_l + 2 * G);              // 128 slots per wave
  int* cnt_l = reinterpret_cast<int*>(pos_all + 4 * 128);
  const int rb = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  uint8_t* pos_l = pos_all + wv * 128;
  // occupied columns [0, OW) and virtual columns [OW, W) of a panel, as 128-bit masks
  const unsigned long long occ0 = OW >= 64 ? ~0ull : ((1ull << OW) - 1ull);
  const unsigned long long occ1 = OW > 64 ? ((OW >= 128) ? ~0ull : ((1ull << (OW - 64)) - 1ull)) : 0ull;
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    const size_t t = (size_t)g * n_rb + rb;
    const ulonglong2 m = actC[t] ? colm[t] : make_ulonglong2(0ull, 0ull);
    cm_l[2 * g] = m.x;
    cm_l[2 * g + 1] = m.y;
  }
  // work counting (wcnt != NULL): per block and row block, the nonzeros of the touched columns
  // before the block (read and written: 16 bytes each) and 6 flops per rotation and row of
  // their union
  unsigned long long w_flops = 0, w_bytes = 0;
  __syncthreads();
  for (int r = 0; r < n_rounds; ++r) {
    const int b0 = roff[r], b1 = roff[r + 1];
    for (int c0 = b0; c0 < b1; c0 += 256) {
      // every thread checks one rotating block of the round; the relevant ones go to LDS
      const int4 mt = (c0 + (int)threadIdx.x < b1) ? meta[c0 + threadIdx.x] : make_int4(-1, 0, 0, 0);
      if (threadIdx.x == 0) cnt_l[0] = 0;
      __syncthreads();
      bool rel = false;
      if (mt.x >= 0) {
        const ulonglong2 tm = tmask[mt.x];
        rel = ((cm_l[2 * mt.y] & tm.x & occ0) | (cm_l[2 * mt.y + 1] & tm.y & occ1) |
               (cm_l[2 * mt.z] & tm.x & ~occ0) | (cm_l[2 * mt.z + 1] & tm.y & ~occ1)) != 0ull;
      }
      const unsigned long long m = __ballot(rel);
      int off = 0;
      if (lane == 0 && m) off = atomicAdd(cnt_l, __popcll(m));
      off = __shfl(off, 0);
      if (rel) list_l[off + __popcll(m & ((1ull << lane) - 1ull))] = mt;
      __syncthreads();
      const int nl = cnt_l[0];
      // a wave's next block: its touched columns and tile slots load while this one is applied
      int4 itn = make_int4(0, 0, 0, 0);
      int tcl0n = 0, tcl1n = 0, sgin = -1, shin = -1;
      auto fetch = [&](int en) {
        itn = list_l[en];
        const int* tcn = tcol + (size_t)itn.x * W;
        tcl0n = (lane < itn.w) ? tcn[lane] : 0;
        tcl1n = (lane + 64 < itn.w) ? tcn[lane + 64] : 0;
        sgin = slot[(size_t)itn.y * n_rb + rb];
        shin = slot[(size_t)itn.z * n_rb + rb];
      };
      if (wv < nl) fetch(wv);
      for (int e = wv; e < nl; e += nw) {
        const int4 it = itn;
        const int tcl0 = tcl0n, tcl1 = tcl1n, sgi = sgin, shi = shin;
        if (e + nw < nl) fetch(e + nw);
        const int b = it.x, g = it.y, h = it.z, T = it.w;
        const int nt_n = (T + 15) >> 4;
        const Real* Rb = R + (size_t)b * W * W;
        // a tile without a slot is all zero and stays so: its columns are never nonzero in
        // cm_l, so nothing is gathered from it; a nonzero written to it is a capacity error
        double* Cg = C + (size_t)(sgi < 0 ? 0 : sgi) * RB * W;
        double* Ch = C + (size_t)(shi < 0 ? 0 : shi) * RB * W;
        // touched columns (two per lane) and whether each is nonzero at rb; the nonzero ones'
        // positions, packed in order, form the K dimension
        auto col_nz = [&](int col) {
          const int grp = col < OW ? g : h;
          return (cm_l[2 * grp + (col >> 6)] >> (col & 63)) & 1ull;
        };
        const bool nz0 = lane < T && col_nz(tcl0);
        const bool nz1 = lane + 64 < T && col_nz(tcl1);
        const unsigned long long q0 = __ballot(nz0), q1 = __ballot(nz1);
        const unsigned long long below = (1ull << lane) - 1ull;
        const int n0 = __popcll(q0);
        if (nz0) pos_l[__popcll(q0 & below)] = (uint8_t)lane;
        if (nz1) pos_l[n0 + __popcll(q1 & below)] = (uint8_t)(lane + 64);
        const int nzk = n0 + __popcll(q1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        acc_t acc[NTMAX];
#pragma unroll
        for (int n = 0; n < NTMAX; ++n) acc[n] = acc_t{0, 0, 0, 0};
        unsigned int w_rows = 0u, w_nnz = 0u;
        for (int s0 = 0; s0 < nzk; s0 += 16) {
          // four k-steps: packed slots s0 + 4 u + lk, gathers all in flight together
          Real a[4];
          int kp[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int slot = s0 + 4 * u + lk;
            const bool in = slot < nzk;
            const int k = in ? pos_l[slot] : 0;
            const int c0 = __shfl(tcl0, k & 63), c1 = __shfl(tcl1, k & 63);
            const int col = (k < 64) ? c0 : c1;
            kp[u] = k;
            a[u] = in ? (Real)((col < OW ? Cg : Ch)[lr * W + col]) : Real(0);
          }
          if (wcnt) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const unsigned long long bb = __ballot(a[u] != Real(0));      // bit = 16 lk + row
              w_nnz += __popcll(bb);
              w_rows |= (unsigned int)((bb | (bb >> 16) | (bb >> 32) | (bb >> 48)) & 0xffffull);
            }
          }
#pragma unroll
          for (int n = 0; n < NTMAX; ++n) {
            if (n >= nt_n) break;
            Real rv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) rv[u] = Rb[(size_t)kp[u] * W + n * 16 + lr];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (s0 + 4 * u < nzk) acc[n] = Mfma<Real>::op(a[u], rv[u], acc[n]);
          }
        }
        // write back with the cut |C| < eps; the written columns' new nonzero bits
        unsigned long long ng0 = 0, ng1 = 0, nh0 = 0, nh1 = 0;
#pragma unroll
        for (int n = 0; n < NTMAX; ++n) {
          const int j = n * 16 + lr;
          const int c0 = __shfl(tcl0, j & 63), c1 = __shfl(tcl1, j & 63);
          int nzc = 0;
          const int col = (j < 64) ? c0 : c1;
          if (n < nt_n && j < T) {
            double* base = (col < OW) ? Cg : Ch;
            const bool has = (col < OW) ? sgi >= 0 : shi >= 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              double x = (double)acc[n][q];
              if (fabs(x) < eps) x = 0.0;
              if (has) {
                base[Mfma<Real>::row(lk, q) * W + col] = x;
                nzc |= x != 0.0;
              } else if (x != 0.0) {
                note_capacity(cap_err, (size_t)((col < OW) ? g : h) * n_rb + rb);
              }
            }
          }
          nzc |= __shfl_xor(nzc, 16);
          nzc |= __shfl_xor(nzc, 32);
          if (nzc && lk == 0) {
            const unsigned long long bit = 1ull << (col & 63);
            if (col < OW) { if (col < 64) ng0 |= bit; else ng1 |= bit; }
            else { if (col < 64) nh0 |= bit; else nh1 |= bit; }
          }
        }
        for (int o = 32; o > 0; o >>= 1) {
          ng0 |= __shfl_xor(ng0, o);
          ng1 |= __shfl_xor(ng1, o);
          nh0 |= __shfl_xor(nh0, o);
          nh1 |= __shfl_xor(nh1, o);
        }
        if (lane == 0) {
          // another block of the round may change the other half (virtual / occupied) of the
          // same group's bits: disjoint bits, atomic updates
          const ulonglong2 tm = tmask[b];
          atomicAnd(&cm_l[2 * g], ~(tm.x & occ0));
          atomicAnd(&cm_l[2 * g + 1], ~(tm.y & occ1));
          if (ng0) atomicOr(&cm_l[2 * g], ng0);
          if (ng1) atomicOr(&cm_l[2 * g + 1], ng1);
          atomicAnd(&cm_l[2 * h], ~(tm.x & ~occ0));
          atomicAnd(&cm_l[2 * h + 1], ~(tm.y & ~occ1));
          if (nh0) atomicOr(&cm_l[2 * h], nh0);
          if (nh1) atomicOr(&cm_l[2 * h + 1], nh1);
        }
        if (wcnt) {
          w_bytes += 16ull * w_nnz;
          w_flops += 6ull * (unsigned long long)rot_cnt[b] * (unsigned long long)__popc(w_rows);
        }
      }
      __syncthreads();
    }
  }
  // exact flags of the row block's tiles
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    const size_t t = (size_t)g * n_rb + rb;
    const unsigned long long m0 = cm_l[2 * g], m1 = cm_l[2 * g + 1];
    unsigned int sl = 0u;
    for (int n = 0; n < 8; ++n)
      if (((n < 4 ? m0 : m1) >> (16 * (n & 3))) & 0xffffull) sl |= 1u << n;
    actC[t] = (uint8_t)(sl != 0u);
    cmask[t] = sl;
    colm[t] = make_ulonglong2(m0, m1);
  }
  if (wcnt && lane == 0) {
    if (w_flops) atomicAdd(wcnt, w_flops);
    if (w_bytes) atomicAdd(wcnt + 1, w_bytes);
  }
}

void launch_givens_rb(const View& v, int n_rounds, const int* roff, const int4* meta, const ulonglong2* tmask,
                      const int* tcol, const double* R, const float* R32, double eps, double* C, uint8_t* actC,
                      unsigned int* cmask, ulonglong2* colm, const int* rot_cnt, unsigned long long* wcnt,
                      hipStream_t s) {
  if (n_rounds <= 0) return;
  const size_t lds = 256 * sizeof(int4) + 2 * sizeof(unsigned long long) * (size_t)v.G + 4 * 128 + 16;
  switch ((v.W + 15) / 16) {
#define SSCF_GIV(N) case N: \
    if (R32) hipLaunchKernelGGL((k_givens_rb<N, float>), dim3(v.n_rb), dim3(256), lds, s, v.G, v.n_rb, v.W, v.OW, n_rounds, roff, meta, tmask, tcol, R32, eps, v.slot, C, actC, cmask, colm, rot_cnt, v.cap_err, wcnt); \
    else hipLaunchKernelGGL((k_givens_rb<N, double>), dim3(v.n_rb), dim3(256), lds, s, v.G, v.n_rb, v.W, v.OW, n_rounds, roff, meta, tmask, tcol, R, eps, v.slot, C, actC, cmask, colm, rot_cnt, v.cap_err, wcnt); \
    break;
    SSCF_GIV(1) SSCF_GIV(2) SSCF_GIV(3) SSCF_GIV(4) SSCF_GIV(5) SSCF_GIV(6) SSCF_GIV(7) SSCF_GIV(8)
#undef SSCF_GIV
  }
}

// ---------------------------------------------------------------------------------------
// Mulliken charges (section 3.7, eq. pop): q_a = sum_{u in a} 2 sum_{i occ} C_ui (S C)_ui.
// Y holds S C of the C before its last normalization, so (S C)_ui = Y_ui / sc_i.
// Row sums are formed panel by panel in increasing order (fixed order).
// ---------------------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_charges_rows(int G, int n_rb, int n_ao, int W, const int* slot,
                                                      const int* slotY, const double* C,
                                                      const int* listTC, const int* cntTC, const double* Y,
                                                      const uint8_t* actY, const double* sc, const int* pnocc,
                                                      double* rowq) {
  __shared__ int s_g[256], s_so[256], s_sy[256], s_no[256];
  const int rb = blockIdx.x;
  const int k = threadIdx.x >> 4, l = threadIdx.x & 15;
  double acc = 0.0;
  const int* LC = listTC + (size_t)rb * G;
  const int nc = cntTC[rb];
  for (int i0 = 0; i0 < nc; i0 += 256) {         // the groups active in C at rb, ascending
    // their slots and occupied counts, 256 at a time, one group per thread (no = 0: skipped)
    {
      const int i = i0 + (int)threadIdx.x;
      int g = 0, so = 0, sy = 0, no = 0;
      if (i < nc) {
        g = LC[i];
        const size_t tile = (size_t)g * n_rb + rb;
        if (actY[tile]) {
          so = slot[tile];
          sy = slotY[tile];
          no = pnocc[g];
        }
      }
      s_g[threadIdx.x] = g;
      s_so[threadIdx.x] = so;
      s_sy[threadIdx.x] = sy;
      s_no[threadIdx.x] = no;
    }
    __syncthreads();
    const int nb = nc - i0 < 256 ? nc - i0 : 256;
    for (int j = 0; j < nb; ++j) {
      const int no = s_no[j];
      if (!no) continue;
      const double* Cr = C + ((size_t)s_so[j] * RB + k) * W;
      const double* Yr = Y + ((size_t)s_sy[j] * RB + k) * W;
      const double* s = sc + (size_t)s_g[j] * W;
      double part = 0.0;
      for (int c = l; c < no; c += 16) part += Cr[c] * Yr[c] / s[c];
      for (int o = 8; o > 0; o >>= 1) part += __shfl_xor(part, o, 16);
      acc += part;
    }
    __syncthreads();
  }
  const int mu = rb * RB + k;
  if (l == 0 && mu < n_ao) rowq[mu] = 2.0 * acc;
}
void launch_charges_rows(const View& v, const double* C, const int* listTC, const int* cntTC, const double* Y,
                         const uint8_t* actY, const double* sc, const int* pnocc, double* rowq, hipStream_t s) {
  hipLaunchKernelGGL(k_charges_rows, dim3(v.n_rb), dim3(256), 0, s, v.G, v.n_rb, v.n_ao, v.W, v.slot, v.slotY, C,
                     listTC, cntTC, Y, actY, sc, pnocc, rowq);
}

__global__ void k_atom_charges(int n_atoms, const int64_t* ao_off, const double* rowq, const double* q0, double* q,
                               double* q_prev, double* dq, Scalars* sd, int shift_prev) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0;
  if (a < n_atoms) {
    double s = 0.0;
    for (int64_t mu = ao_off[a]; mu < ao_off[a + 1]; ++mu) s += rowq[mu];
    const double old = q[a];
    if (shift_prev) { q_prev[a] = old; d = fabs(s - old); }
    q[a] = s;
    dq[a] = s - q0[a];
  }
  block_max_to(d, &sd->dq_bits);
}
void launch_atom_charges(const View& v, const int64_t* ao_off, const double* rowq, double* q, double* q_prev,
                         double* dq, Scalars* sd, int shift_prev, hipStream_t s) {
  hipLaunchKernelGGL(k_atom_charges, dim3(nblk(v.n_atoms, 256)), dim3(256), 0, s, v.n_atoms, ao_off, rowq, v.q0, q,
                     q_prev, dq, sd, shift_prev);
}

// ---------------------------------------------------------------------------------------
// energy sums (FP64, Neumaier compensation, fixed order)
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ void nm_add(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

// E_band = 2 sum_{i occ} C_i^T H0 C_i from the per-column dots d[g][c]
__global__ void __launch_bounds__(256) k_sum_band(int G, int W, const double* d, const int* pnocc, Scalars* sd) {
  __shared__ double ss[256], cc[256];
  double s = 0.0, c = 0.0;
  for (int g = threadIdx.x; g < G; g += 256)
    for (int j = 0; j < pnocc[g]; ++j) nm_add(s, c, d[(size_t)g * W + j]);
  ss[threadIdx.x] = s;
  cc[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0, Cc = 0.0;
    for (int i = 0; i < 256; ++i) { nm_add(S, Cc, ss[i]); nm_add(S, Cc, cc[i]); }
    sd->e_band = 2.0 * (S + Cc);
  }
}
void launch_sum_band(const View& v, const double* d, const int* pnocc, Scalars* sd, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_band, dim3(1), dim3(256), 0, s, v.G, v.W, d, pnocc, sd);
}

__global__ void __launch_bounds__(256) k_sum_coul(int n, int scc, const double* dq, const double* Q, Scalars* sd) {
  __shared__ double ss[256], cc[256];
  double s = 0.0, c = 0.0;
  for (int a = threadIdx.x; a < n; a += 256) nm_add(s, c, 0.5 * dq[a] * Q[a]);
  ss[threadIdx.x] = s;
  cc[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0, Cc = 0.0;
    for (int i = 0; i < 256; ++i) { nm_add(S, Cc, ss[i]); nm_add(S, Cc, cc[i]); }
    sd->e_coul = scc ? (S + Cc) : 0.0;
  }
}
void launch_sum_coul(const View& v, int scc, const double* dq, const double* Q, Scalars* sd, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_coul, dim3(1), dim3(256), 0, s, v.n_atoms, scc, dq, Q, sd);
}

// ---------------------------------------------------------------------------------------
// density on the row-block pattern: P[r][c] = 2 sum_g C_g[r]_occ C_g[c]_occ^T (one wave
// per 16 x 16 block; MFMA over the occupied columns)
// ---------------------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_density_blocks(int nbx, int G, int n_rb, int W, int OW, const int* slot,
                                                        const int* slotB,
                                                        const int* xs_row,
                                                        const int* xs_col, const double* A,
                                                        const unsigned int* cmA, const int* listTA,
                                                        const int* cntTA, const double* B, const uint8_t* actB,
                                                        const unsigned int* cmB, double* P) {
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= nbx) return;
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const int r = xs_row[b], c = xs_col[b];
  d4 acc = d4{0.0, 0.0, 0.0, 0.0};
  const int* LA = listTA + (size_t)r * G;
  const int na = cntTA[r];
  const unsigned int occ = (1u << (OW / 16)) - 1u;
  for (int k = 0; k < na; ++k) {                // the groups active in A at row block r, ascending
    const int g = LA[k];
    const size_t tr = (size_t)g * n_rb + r, tc = (size_t)g * n_rb + c;
    if (!actB[tc]) continue;
    // occupied 16-column slices nonzero on both sides (cmB NULL: B's slices are not tracked);
    // a 4-column k-step that is zero in every lane on either side adds exact zeros
    const unsigned int m = cmA[tr] & (cmB ? cmB[tc] : 0xffffffffu) & occ;
    if (!m) continue;
    const double* At = A + (size_t)slot[tr] * (RB * W) + lr * W + lk;
    const double* Bt = B + (size_t)slotB[tc] * (RB * W) + lr * W + lk;
    for (int sl = 0; sl < OW / 16; ++sl) {
      if (!((m >> sl) & 1u)) continue;
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = At[16 * sl + 4 * u];
        b[u] = Bt[16 * sl + 4 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (__ballot(a[u] != 0.0) && __ballot(b[u] != 0.0)) acc = mfma64(a[u], b[u], acc);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) P[(size_t)b * 256 + (lk + 4 * q) * 16 + lr] = 2.0 * acc[q];
}
// 2 A_occ B_occ^T on the 16 x 16 blocks of the S pattern: the density P (A = B = C) or
// W = 2 C_occ Z_occ^T (B = Z) of the energy gradient
void launch_density_blocks(const View& v, const double* A, const unsigned int* cmA, const int* listTA,
                           const int* cntTA, const double* B, const uint8_t* actB, const unsigned int* cmB,
                           bool B_is_y, double* P, hipStream_t s) {
  hipLaunchKernelGGL(k_density_blocks, dim3((v.nbx + 3) / 4), dim3(256), 0, s, v.nbx, v.G, v.n_rb, v.W, v.OW,
                     v.slot, B_is_y ? v.slotY : v.slot, v.xs_row, v.xs_col, A, cmA, listTA, cntTA, B, actB, cmB, P);
}

// ---------------------------------------------------------------------------------------
// Energy gradient on the pattern of S (atom-block layout of S_val): dE/dX = P and
// dE/dS = -W + 1/2 P (Q_a + Q_b) (the second term only with the charge term of H0), read from
// the 16 x 16 row-block forms of P and W; and dE/d(onsite energy) per atom shell, the sum of
// P over the shell's diagonal (s: the atom's first AO; p: its other AOs).
// ---------------------------------------------------------------------------------------
__global__ void k_grad_assemble(int64_t n, const int64_t* __restrict__ map, const int* __restrict__ xs_row,
                                const int* __restrict__ xs_col, const int* __restrict__ ao_atom,
                                const double* __restrict__ P, const double* __restrict__ Wb,
                                const double* __restrict__ Q, int qterm, double* __restrict__ dX,
                                double* __restrict__ dS) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t e = map[t];
  const int64_t b = e >> 8;
  const int mu = xs_row[b] * RB + (int)((e >> 4) & 15), nu = xs_col[b] * RB + (int)(e & 15);
  const double p = P[e];
  const double qs = qterm ? 0.5 * (Q[ao_atom[mu]] + Q[ao_atom[nu]]) : 0.0;
  dX[t] = p;
  dS[t] = -Wb[e] + p * qs;
}
void launch_grad_assemble(const View& v, int64_t n_val, const int64_t* map, const double* P, const double* Wb,
                          const double* Q, int qterm, double* dX, double* dS, hipStream_t s) {
  if (n_val)
    hipLaunchKernelGGL(k_grad_assemble, dim3(nblk((size_t)n_val, 256)), dim3(256), 0, s, n_val, map, v.xs_row,
                       v.xs_col, v.ao_atom, P, Wb, Q, qterm, dX, dS);
}

__global__ void k_grad_onsite(int n_atoms, const int64_t* __restrict__ ao_off, const int* __restrict__ xs_diag,
                              const double* __restrict__ P, double* __restrict__ out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_atoms) return;
  const int64_t mu0 = ao_off[a];
  double ps = P[(size_t)xs_diag[mu0 / RB] * 256 + (mu0 % RB) * 17], pp = 0.0;
  for (int64_t mu = mu0 + 1; mu < ao_off[a + 1]; ++mu) pp += P[(size_t)xs_diag[mu / RB] * 256 + (mu % RB) * 17];
  out[2 * a] = ps;
  out[2 * a + 1] = pp;
}
void launch_grad_onsite(const View& v, const int64_t* ao_off, const int* xs_diag, const double* P, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_grad_onsite, dim3(nblk(v.n_atoms, 256)), dim3(256), 0, s, v.n_atoms, ao_off, xs_diag, P, out);
}

// ---------------------------------------------------------------------------------------
// Energy gradient (differentiation form): Z_g[r] = sum_{h ~ g} C_h,occ[r] F(h, g) with
// F(h, g) = C_h,occ^T H C_g,occ (OW x OW; FA holds the blocks with rows = MOs of pg[p],
// FB those with rows = MOs of ph[p]).  One wave per output tile, occupied columns only; Z lives
// in the pool of Y.
// ---------------------------------------------------------------------------------------
template <int NO>
__global__ void __launch_bounds__(256) k_apply_occ(int G, int n_rb, int W, int nchunk, const int* __restrict__ slot,
                                                   const int* __restrict__ slotZ, const double* __restrict__ C,
                                                   const uint8_t* __restrict__ actC,
                                                   const unsigned int* __restrict__ cmask, const int* __restrict__ gn_ptr,
                                                   const int* __restrict__ gn, const int* __restrict__ pair_of,
                                                   const int* __restrict__ pg, const double* __restrict__ FA,
                                                   const double* __restrict__ FB, const int* __restrict__ listZ,
                                                   const int* __restrict__ cntZ, double* __restrict__ Z) {
  constexpr int OW = NO * 16;
  int chunk;
  const int g = xcd_group_chunk(nchunk, chunk);
  if (g >= G) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = chunk * 4 + wv;
  if (t >= cntZ[g]) return;
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const int r = listZ[(size_t)g * n_rb + t];
  d4 acc[NO];
#pragma unroll
  for (int n = 0; n < NO; ++n) acc[n] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k = gn_ptr[g]; k < gn_ptr[g + 1]; ++k) {
    const int h = gn[k];
    const size_t th = (size_t)h * n_rb + r;
    if (!actC[th]) continue;
    // the occupied 16-column slices of C_h(r) that hold a nonzero; a 4-column k-step that is
    // zero in every lane adds exact zeros and is skipped
    const unsigned int m = cmask[th] & ((1u << NO) - 1u);
    if (!m) continue;
    const int p = pair_of[(size_t)g * G + h];
    const double* Fp = ((pg[p] == h) ? FA : FB) + (size_t)p * OW * OW + lr;
    const double* Ch = C + (size_t)slot[th] * (RB * W) + lr * W + lk;
    for (int sl = 0; sl < NO; ++sl) {
      if (!((m >> sl) & 1u)) continue;
      double a[4], f[4][NO];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int s = 4 * sl + u;
        a[u] = Ch[4 * s];
#pragma unroll
        for (int n = 0; n < NO; ++n) f[u][n] = Fp[(4 * s + lk) * OW + n * 16];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (__ballot(a[u] != 0.0))
#pragma unroll
          for (int n = 0; n < NO; ++n) acc[n] = mfma64(a[u], f[u][n], acc[n]);
    }
  }
  double* Zt = Z + (size_t)slotZ[(size_t)g * n_rb + r] * (RB * W);
#pragma unroll
  for (int n = 0; n < NO; ++n)
#pragma unroll
    for (int q = 0; q < 4; ++q) Zt[(lk + 4 * q) * W + n * 16 + lr] = acc[n][q];
}

void launch_apply_occ(const View& v, const double* C, const uint8_t* actC, const unsigned int* cmask,
                      const int* gn_ptr, const int* gn,
                      const int* pair_of, const int* pg, const double* FA, const double* FB, const int* listZ,
                      const int* cntZ, double* Z, hipStream_t s) {
  const int nchunk = (v.max_y + 3) / 4;
  dim3 grid(xcd_grid(v.G, nchunk)), blk(256);
  switch (v.OW / 16) {
#define SSCF_APO(NO) case NO: hipLaunchKernelGGL(k_apply_occ<NO>, grid, blk, 0, s, v.G, v.n_rb, v.W, nchunk, v.slot, v.slotY, C, actC, cmask, gn_ptr, gn, pair_of, pg, FA, FB, listZ, cntZ, Z); break;
    SSCF_APO(1) SSCF_APO(2) SSCF_APO(3) SSCF_APO(4) SSCF_APO(5) SSCF_APO(6) SSCF_APO(7) SSCF_APO(8)
#undef SSCF_APO
    default: break;
  }
}

// ---------------------------------------------------------------------------------------
// FP32 form of C^T H C (the paper already runs this product in single precision, §4.1):
// Y32 = H32 C32 and the occupied-virtual blocks and diagonal of C32^T Y32, FP32 matrix cores
// with FP32 accumulation.  C itself stays FP64; C32 is its rounding to FP32, made once per
// step for the active tiles (k_round_c32), so every product reads half the bytes.
// ---------------------------------------------------------------------------------------

// (only the nonzero 16-column slices: the FP32 kernels read no other slice of C32)
__global__ void __launch_bounds__(256) k_round_c32(int n_rb, int W, const int* __restrict__ slot,
                                                   const double* __restrict__ C,
                                                   const int* __restrict__ list, const int* __restrict__ cnt,
                                                   const unsigned int* __restrict__ cmask,
                                                   float* __restrict__ C32) {
  const int g = blockIdx.y;
  for (int t = blockIdx.x; t < cnt[g]; t += gridDim.x) {
    const size_t tile = (size_t)g * n_rb + list[(size_t)g * n_rb + t];
    const size_t base = (size_t)slot[tile] * (size_t)(RB * W);
    const unsigned int cm = cmask[tile];
    for (int e = threadIdx.x; e < RB * W; e += 256)
      if ((cm >> ((e % W) >> 4)) & 1u) C32[base + e] = (float)C[base + e];
  }
}
void launch_round_c32(const View& v, const double* C, const int* list, const int* cnt, const unsigned int* cmask,
                      float* C32, hipStream_t s) {
  hipLaunchKernelGGL(k_round_c32, dim3(std::min(v.n_rb, TILE_STRIDE_WG), v.G), dim3(256), 0, s, v.n_rb, v.W, v.slot,
                     C, list, cnt, cmask, C32);
}

template <int MW, int NW>
__global__ void __launch_bounds__(256) k_pair32(int n_rb, int W, const int* __restrict__ slot,
                                                const int* __restrict__ slotY,
                                                const int* __restrict__ perm, int maxc,
                                                const int* __restrict__ pg, const int* __restrict__ ph,
                                                const float* __restrict__ C, const int* __restrict__ listC,
                                                const int* __restrict__ cntC, const unsigned int* __restrict__ cmask,
                                                const float* __restrict__ Y, const uint8_t* __restrict__ actY,
                                                const unsigned int* __restrict__ ymask, int row_off, int MT,
                                                int col_off, int NT, double* __restrict__ out, int ld,
                                                size_t out_stride, unsigned long long* ctr) {
  const int p = xcd_item(perm, maxc);
  if (p < 0) return;
  const int g = pg[p], h = ph[p];
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int MH = (MT + 1) / 2, NH = (NT + 1) / 2;
  const int mt0 = (w >> 1) * MH, nt0 = (w & 1) * NH;
  const int mc = min(MH, MT - mt0), nc = min(NH, NT - nt0);
  f4 acc[MW][NW];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const size_t gb = (size_t)g * n_rb, hb = (size_t)h * n_rb;
  const int cnt = cntC[g];
  unsigned int n_mfma = 0;
  if (mc > 0 && nc > 0) {
    const unsigned int mcm = (1u << mc) - 1u, ncm = (1u << nc) - 1u;
    const int sa = row_off / 16 + mt0, sb = col_off / 16 + nt0;
    // the rows active in both panels, 64 at a time, with their slice masks, before any product
    for (int base = 0; base < cnt; base += 64) {
      const int t = base + lane;
      int rr = 0, sc = 0, sy = 0;
      unsigned int mab = 0u;
      if (t < cnt) {
        rr = listC[gb + t];
        if (actY[hb + rr]) {
          const unsigned int ma = (cmask[gb + rr] >> sa) & mcm, mb = (ymask[hb + rr] >> sb) & ncm;
          if (ma && mb) {
            mab = ma | (mb << 16);
            sc = slot[gb + rr];                // the common rows' slots in one round trip
            sy = slotY[hb + rr];
          }
        }
      }
      unsigned long long m = __ballot(mab != 0u);
      while (m) {
        const int j = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const unsigned int mj = __builtin_amdgcn_readfirstlane(__shfl((int)mab, j));
        const unsigned int ma = mj & 0xffffu, mb = mj >> 16;
        const size_t scj = (size_t)(unsigned int)__builtin_amdgcn_readfirstlane(__shfl(sc, j));
        const size_t syj = (size_t)(unsigned int)__builtin_amdgcn_readfirstlane(__shfl(sy, j));
        const float* Ct = C + scj * (RB * W) + row_off + mt0 * 16 + lr;
        const float* Yt = Y + syj * (RB * W) + col_off + nt0 * 16 + lr;
        float a[4][MW], b[4][NW];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int ro = (4 * s + lk) * W;
#pragma unroll
          for (int i = 0; i < MW; ++i) a[s][i] = (ma & (1u << i)) ? Ct[ro + i * 16] : 0.f;
#pragma unroll
          for (int jj = 0; jj < NW; ++jj) b[s][jj] = (mb & (1u << jj)) ? Yt[ro + jj * 16] : 0.f;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int i = 0; i < MW; ++i)
#pragma unroll
            for (int jj = 0; jj < NW; ++jj)
              if ((ma & (1u << i)) && (mb & (1u << jj))) {
                acc[i][jj] = mfma32(a[s][i], b[s][jj], acc[i][jj]);
                ++n_mfma;
              }
      }
    }
  }
  double* o = out + (size_t)p * out_stride;
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j)
      if (i < mc && j < nc)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          o[(size_t)((mt0 + i) * 16 + 4 * lk + q) * ld + (nt0 + j) * 16 + lr] = (double)acc[i][j][q];
  if (ctr && lane == 0 && n_mfma) atomicAdd(ctr, (unsigned long long)n_mfma);
}

void launch_pair32(const View& v, int n_pairs, const int* perm, int maxc, const int* pg, const int* ph,
                   const float* C, const int* listC,
                   const int* cntC, const unsigned int* cmask, const float* Y, const uint8_t* actY,
                   const unsigned int* ymask, int row_off, int MT, int col_off, int NT, double* out, int ld,
                   size_t out_stride, unsigned long long* ctr, hipStream_t s) {
  if (n_pairs <= 0) return;
  const int mw = (MT + 1) / 2, nw = (NT + 1) / 2;
  const int m = mw > nw ? mw : nw;
  dim3 grid(N_XCD * maxc), blk(256);
  if (m <= 1)
    hipLaunchKernelGGL((k_pair32<1, 1>), grid, blk, 0, s, v.n_rb, v.W, v.slot, v.slotY, perm, maxc, pg, ph, C, listC, cntC, cmask, Y, actY, ymask, row_off, MT, col_off, NT, out, ld, out_stride, ctr);
  else if (m <= 2)
    hipLaunchKernelGGL((k_pair32<2, 2>), grid, blk, 0, s, v.n_rb, v.W, v.slot, v.slotY, perm, maxc, pg, ph, C, listC, cntC, cmask, Y, actY, ymask, row_off, MT, col_off, NT, out, ld, out_stride, ctr);
  else if (m <= 3)
    hipLaunchKernelGGL((k_pair32<3, 3>), grid, blk, 0, s, v.n_rb, v.W, v.slot, v.slotY, perm, maxc, pg, ph, C, listC, cntC, cmask, Y, actY, ymask, row_off, MT, col_off, NT, out, ld, out_stride, ctr);
  else
    hipLaunchKernelGGL((k_pair32<4, 4>), grid, blk, 0, s, v.n_rb, v.W, v.slot, v.slotY, perm, maxc, pg, ph, C, listC, cntC, cmask, Y, actY, ymask, row_off, MT, col_off, NT, out, ld, out_stride, ctr);
}

__global__ void __launch_bounds__(256) k_coldot32(int n_rb, int W, const int* slot, const int* slotY, const float* C,
                                                  const int* listC, const int* cntC, const unsigned int* cmask,
                                                  const float* Y, const uint8_t* actY, double* out) {
  __shared__ int s_so[256], s_sy[256];
  __shared__ unsigned int s_cm[256];
  const int g = blockIdx.x, c = threadIdx.x;
  const size_t gb = (size_t)g * n_rb;
  const int cnt = cntC[g];
  float s = 0.f;
  for (int i0 = 0; i0 < cnt; i0 += blockDim.x) {
    const int nb = stage_tiles(gb, listC, i0, 1, cnt - i0, slot, slotY, cmask, actY, s_so, s_sy, s_cm);
    if (c < W)
      for (int j = 0; j < nb; ++j) {
        if (!((s_cm[j] >> (c >> 4)) & 1u)) continue;   // a zero slice adds zeros
        const float* Ct = C + (size_t)s_so[j] * (RB * W) + c;
        const float* Yt = Y + (size_t)s_sy[j] * (RB * W) + c;
#pragma unroll
        for (int k = 0; k < RB; ++k) s += Ct[k * W] * Yt[k * W];
      }
    __syncthreads();
  }
  if (c < W) out[(size_t)g * W + c] = (double)s;
}
void launch_coldot32(const View& v, const float* C, const int* listC, const int* cntC, const unsigned int* cmask,
                     const float* Y, const uint8_t* actY, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_coldot32, dim3(v.G), dim3(v.W <= 64 ? 64 : (v.W <= 128 ? 128 : 256)), 0, s, v.n_rb, v.W,
                     v.slot, v.slotY, C, listC, cntC, cmask, Y, actY, out);
}

// ---------------------------------------------------------------------------------------
// Y = X C with one wave per output tile (g, r) and no workgroup synchronization; only the
// 16-column slices in smask are formed (the others are left zero).  A ballot
// over the row's X blocks finds, 64 at a time, those whose C tile is active in panel g, with
// its 16-column slice mask, before any product starts; the wave then streams the products,
// the X block (A operand) and the C tile slices (B operand) read straight from L2 with all
// of a product's loads issued together.  Real as above.
// ---------------------------------------------------------------------------------------
template <int NT, typename Real>
__global__ void __launch_bounds__(256) k_spmm_row(int G, int n_rb, int nchunk, const int* __restrict__ slot,
                                                  const int* __restrict__ slotY, const int* __restrict__ xs_ptr,
                                                  const int* __restrict__ xs_col, const Real* __restrict__ X,
                                                  const Real* __restrict__ C, const uint8_t* __restrict__ actC,
                                                  const unsigned int* __restrict__ cmask,
                                                  const int* __restrict__ listY, const int* __restrict__ cntY,
                                                  Real* __restrict__ Y, unsigned int* __restrict__ ymask,
                                                  unsigned int smask, unsigned long long* ctr) {
  constexpr int W = NT * 16;
  typedef typename Mfma<Real>::acc_t acc_t;
  int chunk;
  const int g = xcd_group_chunk(nchunk, chunk);
  if (g >= G) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = chunk * 4 + wv;
  if (t >= cntY[g]) return;
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  const size_t pb = (size_t)g * n_rb;
  const int r = listY[pb + t];
  const int k0 = xs_ptr[r], k1 = xs_ptr[r + 1];
  acc_t acc[NT];
#pragma unroll
  for (int n = 0; n < NT; ++n) acc[n] = acc_t{0, 0, 0, 0};
  unsigned int n_mfma = 0;
  for (int base = k0; base < k1; base += 64) {
    const int k = base + lane;
    int c = 0, sc = 0;
    unsigned int mk = 0u;
    if (k < k1) {
      c = xs_col[k];
      mk = actC[pb + c] ? (cmask[pb + c] & smask) : 0u;
      if (mk) sc = slot[pb + c];               // the products' C slots in one round trip
    }
    unsigned long long m = __ballot(mk != 0u);
    if (!m) continue;
    // X blocks are read once per group and mostly miss L2: the next product's X block is
    // loaded while the current one's C slices load and multiply
    int j = __ffsll((long long)m) - 1;
    m &= m - 1ull;
    Real xn[4];
    {
      const Real* Xb = X + (size_t)(base + j) * 256 + lr * 16 + lk;
#pragma unroll
      for (int s = 0; s < 4; ++s) xn[s] = Xb[4 * s];
    }
    for (;;) {
      const unsigned int mj = __builtin_amdgcn_readfirstlane(__shfl((int)mk, j));
      const size_t scj = (size_t)(unsigned int)__builtin_amdgcn_readfirstlane(__shfl(sc, j));
      Real xa[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) xa[s] = xn[s];
      // k-steps (4 columns of the X block) that hold a nonzero: the others add exact zeros,
      // and their C rows are not read (FP32: their MFMAs still run, on zeros, see below)
      unsigned int km = 0u;
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (__ballot(xa[s] != Real(0))) km |= 1u << s;
      const Real* Ct = C + scj * (RB * W) + lk * W + lr;
      Real cb[4][NT];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int n = 0; n < NT; ++n)
          cb[s][n] = (((mj >> n) & 1u) && ((km >> s) & 1u)) ? Ct[4 * s * W + n * 16] : Real(0);
      int jn = -1;
      if (m) {
        jn = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const Real* Xb = X + (size_t)(base + jn) * 256 + lr * 16 + lk;
#pragma unroll
        for (int s = 0; s < 4; ++s) xn[s] = Xb[4 * s];
      }
      if constexpr (sizeof(Real) == sizeof(double)) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int n = 0; n < NT; ++n)
            if (((mj >> n) & 1u) && ((km >> s) & 1u)) {
              acc[n] = Mfma<Real>::op(xa[s], cb[s][n], acc[n]);
              ++n_mfma;
            }
      } else {
        // FP32: branch-free (a masked slice is zero); branches around FP32 MFMAs make the
        // compiler move the accumulators between register files at every join
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int n = 0; n < NT; ++n) acc[n] = Mfma<Real>::op(xa[s], cb[s][n], acc[n]);
        n_mfma += 4 * NT;
      }
      if (jn < 0) break;
      j = jn;
    }
  }
  Real* Yt = Y + (size_t)slotY[pb + r] * (RB * W);
  unsigned int ym = 0;
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    int nz = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Yt[Mfma<Real>::row(lk, q) * W + n * 16 + lr] = acc[n][q];
      nz |= acc[n][q] != Real(0);
    }
    if (__ballot(nz)) ym |= 1u << n;
  }
  if (lane == 0) {
    ymask[pb + r] = ym;
    if (ctr && n_mfma) atomicAdd(ctr, (unsigned long long)n_mfma);
  }
}

template <typename Real>
static void launch_spmm_row(const View& v, const Real* X, const Real* C, const uint8_t* actC,
                            const unsigned int* cmask, const int* listY, const int* cntY, Real* Y,
                            unsigned int* ymask, unsigned int smask, unsigned long long* ctr, hipStream_t s) {
  const int nchunk = (v.max_y + 3) / 4;
  dim3 grid(xcd_grid(v.G, nchunk)), blk(256);
  switch (v.W / 16) {
#define SSCF_SPR(NT) case NT: hipLaunchKernelGGL((k_spmm_row<NT, Real>), grid, blk, 0, s, v.G, v.n_rb, nchunk, v.slot, v.slotY, v.xs_ptr, v.xs_col, X, C, actC, cmask, listY, cntY, Y, ymask, smask, ctr); break;
    SSCF_SPR(1) SSCF_SPR(2) SSCF_SPR(3) SSCF_SPR(4) SSCF_SPR(5) SSCF_SPR(6) SSCF_SPR(7) SSCF_SPR(8)
#undef SSCF_SPR
  }
}

void launch_spmm(const View& v, const double* X, const double* C, const uint8_t* actC, const unsigned int* cmask,
                 const int* listY, const int* cntY, double* Y, unsigned int* ymask, unsigned int smask,
                 unsigned long long* ctr, hipStream_t s) {
  launch_spmm_row<double>(v, X, C, actC, cmask, listY, cntY, Y, ymask, smask, ctr, s);
}

void launch_spmm32(const View& v, const float* X, const float* C, const uint8_t* actC, const unsigned int* cmask,
                   const int* listY, const int* cntY, float* Y, unsigned int* ymask, unsigned long long* ctr,
                   hipStream_t s) {
  launch_spmm_row<float>(v, X, C, actC, cmask, listY, cntY, Y, ymask, 0xffffffffu, ctr, s);
}

}  // namespace sscf
