// Work counting of the sparse SCF passes (SSCF_FLAG_COUNT_WORK).
//
// These kernels measure; none of them changes a value of the method.  They count, on the
// library's own state at the point where each pass runs, the algorithmic work of the pass:
// the multiplications and additions of the sparse operation itself (zero operands do not
// count, whatever tile or padding the kernels use) and each nonzero value read or written
// once.  The definitions are those of sscf_get_kernel_stats in include/sscf.h.  Counting
// launches run between the passes, outside the HIP events that time them.
#include "sscf_internal.h"

namespace sscf {

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// block of 256 threads: sum of v added to *out (one atomic per block).  Every thread of the
// block calls it; the closing barrier keeps a following call's writes to red from overtaking
// thread 0's reads of this one.
__device__ void block_add(unsigned long long v, unsigned long long* out) {
  __shared__ unsigned long long red[4];
  v = wave_sum_u64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long s = red[0] + red[1] + red[2] + red[3];
    if (s) atomicAdd(out, s);
  }
  __syncthreads();
}

// Nonzeros of each AO row of X (16 x 16 blocks on the row-block pattern) into xrow (added;
// zeroed by the caller) and their total into *tot.
template <typename Real>
__global__ void __launch_bounds__(256) k_cnt_xrow(int nbx, const int* __restrict__ xs_row, const Real* __restrict__ X,
                                                  int* __restrict__ xrow, unsigned long long* tot) {
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t b = idx >> 4;
  const int k = (int)(idx & 15);
  int c = 0;
  if (b < (size_t)nbx) {
    const Real* row = X + b * 256 + k * 16;
#pragma unroll
    for (int j = 0; j < 16; ++j) c += row[j] != Real(0);
    if (c) atomicAdd(&xrow[xs_row[b] * RB + k], c);
  }
  block_add((unsigned long long)c, tot);
}

// Over the listed tiles of T: nonzeros in columns [c0, c1) into *nnz; with weight, the sum of
// weight[AO row] over those nonzeros into *wsum; with colnnz, the nonzeros of each column
// (added to colnnz[g W + c]).
template <typename Real>
__global__ void __launch_bounds__(256) k_cnt_tiles(int n_rb, int W, const int* __restrict__ slot, const Real* __restrict__ T,
                                                   const int* __restrict__ list, const int* __restrict__ cnt, int c0,
                                                   int c1, const int* __restrict__ weight, int* __restrict__ colnnz,
                                                   unsigned long long* nnz, unsigned long long* wsum) {
  const int g = blockIdx.y, t = blockIdx.x;
  if (t >= cnt[g]) return;
  const int r = list[(size_t)g * n_rb + t];
  const Real* Tt = T + (size_t)slot[(size_t)g * n_rb + r] * (size_t)(RB * W);
  unsigned long long n = 0, w = 0;
  for (int e = threadIdx.x; e < RB * W; e += 256) {
    const int c = e % W, k = e / W;
    if (c < c0 || c >= c1 || Tt[e] == Real(0)) continue;
    ++n;
    if (weight) w += (unsigned long long)weight[r * RB + k];
    if (colnnz) atomicAdd(&colnnz[(size_t)g * W + c], 1);
  }
  block_add(n, nnz);
  if (wsum) block_add(w, wsum);
}

// Row masks of the listed tiles: masks[(slot * 16 + k)] = the nonzero columns of row k (slot of
// the pool T lives in)
// (bit c of .x for c < 64, bit c - 64 of .y).  One wave per tile.
template <typename Real>
__global__ void __launch_bounds__(64) k_row_masks(int n_rb, int W, const int* __restrict__ slot, const Real* __restrict__ T,
                                                  const int* __restrict__ list, const int* __restrict__ cnt,
                                                  ulonglong2* __restrict__ masks) {
  const int g = blockIdx.y, t = blockIdx.x;
  if (t >= cnt[g]) return;
  const size_t sl = (size_t)slot[(size_t)g * n_rb + list[(size_t)g * n_rb + t]];
  const Real* Tt = T + sl * (size_t)(RB * W);
  const int lane = threadIdx.x;
  for (int k = 0; k < RB; ++k) {
    const unsigned long long lo = __ballot(lane < W && Tt[k * W + lane] != Real(0));
    const unsigned long long hi = __ballot(lane + 64 < W && Tt[k * W + lane + 64] != Real(0));
    if (lane == 0) masks[sl * RB + k] = make_ulonglong2(lo, hi);
  }
}

__device__ __forceinline__ unsigned long long range_bits(int lo, int hi, int word) {
  // bits [lo, hi) of the 128-bit column range restricted to 64-bit word `word`
  const int a = max(lo - 64 * word, 0), b = min(hi - 64 * word, 64);
  if (b <= a) return 0ull;
  const unsigned long long upto = (b == 64) ? ~0ull : ((1ull << b) - 1ull);
  return upto & ~((1ull << a) - 1ull);
}

// Pair products C_g^T Y_h: for every item (g = ig[i], h = ih[i]) and every row active in both,
// the number of (column a of g in [a0, a1), column b of h in [b0, b1)) with both entries
// nonzero; with tri (self pairs of C^T S C) only a <= b.  Sum into *out.  One wave per item.
__global__ void __launch_bounds__(64) k_cnt_pairs(int n_items, int n_rb, const int* __restrict__ slot,
                                                  const int* __restrict__ slotY, const int* __restrict__ ig,
                                                  const int* __restrict__ ih, const int* __restrict__ listC,
                                                  const int* __restrict__ cntC, const uint8_t* __restrict__ actY,
                                                  const ulonglong2* __restrict__ mC, const ulonglong2* __restrict__ mY,
                                                  int a0, int a1, int b0, int b1, int tri, unsigned long long* out) {
  const int i = blockIdx.x;
  if (i >= n_items) return;
  const int g = ig[i], h = ih[i];
  const bool self = tri && g == h;
  const unsigned long long ra0 = range_bits(a0, a1, 0), ra1 = range_bits(a0, a1, 1);
  const unsigned long long rb0 = range_bits(b0, b1, 0), rb1 = range_bits(b0, b1, 1);
  unsigned long long s = 0;
  for (int t = threadIdx.x; t < cntC[g]; t += 64) {
    const int r = listC[(size_t)g * n_rb + t];
    if (!actY[(size_t)h * n_rb + r]) continue;
    const ulonglong2* pc = mC + (size_t)slot[(size_t)g * n_rb + r] * RB;
    const ulonglong2* py = mY + (size_t)slotY[(size_t)h * n_rb + r] * RB;
    for (int k = 0; k < RB; ++k) {
      const unsigned long long c0 = pc[k].x & ra0, c1 = pc[k].y & ra1;
      const unsigned long long y0 = py[k].x & rb0, y1 = py[k].y & rb1;
      if (!self) {
        s += (unsigned long long)(__popcll(c0) + __popcll(c1)) * (unsigned long long)(__popcll(y0) + __popcll(y1));
        continue;
      }
      for (unsigned long long m = y0; m; m &= m - 1ull) {
        const int j = __ffsll((long long)m) - 1;
        s += __popcll(c0 & ((2ull << j) - 1ull));
      }
      for (unsigned long long m = y1; m; m &= m - 1ull) {
        const int j = __ffsll((long long)m) - 1;
        s += __popcll(c0) + __popcll(c1 & ((2ull << j) - 1ull));
      }
    }
  }
  s = wave_sum_u64(s);
  if (threadIdx.x == 0 && s) atomicAdd(out, s);
}

// sum_c a[c] b[c] and sum_c b[c] over n entries
__global__ void __launch_bounds__(256) k_cnt_dot(size_t n, const int* __restrict__ a, const int* __restrict__ b,
                                                 unsigned long long* dot, unsigned long long* sumb) {
  unsigned long long d = 0, s = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    d += (unsigned long long)a[i] * (unsigned long long)b[i];
    s += (unsigned long long)b[i];
  }
  block_add(d, dot);
  block_add(s, sumb);
}

static inline unsigned int cgrid(size_t n, int t) { return (unsigned int)((n + t - 1) / t); }

void launch_cnt_xrow(const View& v, const void* X, bool fp32, int* xrow, unsigned long long* tot, hipStream_t s) {
  const size_t n = (size_t)v.nbx * RB;
  if (fp32)
    hipLaunchKernelGGL(k_cnt_xrow<float>, dim3(cgrid(n, 256)), dim3(256), 0, s, v.nbx, v.xs_row, (const float*)X,
                       xrow, tot);
  else
    hipLaunchKernelGGL(k_cnt_xrow<double>, dim3(cgrid(n, 256)), dim3(256), 0, s, v.nbx, v.xs_row, (const double*)X,
                       xrow, tot);
}

void launch_cnt_tiles(const View& v, const void* T, bool fp32, bool is_y, const int* list, const int* cnt, int c0,
                      int c1, const int* weight, int* colnnz, unsigned long long* nnz, unsigned long long* wsum,
                      hipStream_t s) {
  const int* sl = is_y ? v.slotY : v.slot;
  if (fp32)
    hipLaunchKernelGGL(k_cnt_tiles<float>, dim3(v.n_rb, v.G), dim3(256), 0, s, v.n_rb, v.W, sl, (const float*)T, list,
                       cnt, c0, c1, weight, colnnz, nnz, wsum);
  else
    hipLaunchKernelGGL(k_cnt_tiles<double>, dim3(v.n_rb, v.G), dim3(256), 0, s, v.n_rb, v.W, sl, (const double*)T, list,
                       cnt, c0, c1, weight, colnnz, nnz, wsum);
}

void launch_row_masks(const View& v, const void* T, bool fp32, bool is_y, const int* list, const int* cnt,
                      ulonglong2* masks, hipStream_t s) {
  const int* sl = is_y ? v.slotY : v.slot;
  if (fp32)
    hipLaunchKernelGGL(k_row_masks<float>, dim3(v.n_rb, v.G), dim3(64), 0, s, v.n_rb, v.W, sl, (const float*)T, list,
                       cnt, masks);
  else
    hipLaunchKernelGGL(k_row_masks<double>, dim3(v.n_rb, v.G), dim3(64), 0, s, v.n_rb, v.W, sl, (const double*)T, list,
                       cnt, masks);
}

void launch_cnt_pairs(const View& v, int n_items, const int* ig, const int* ih, const int* listC, const int* cntC,
                      const uint8_t* actY, const ulonglong2* mC, const ulonglong2* mY, int a0, int a1, int b0,
                      int b1, int tri, unsigned long long* out, hipStream_t s) {
  if (n_items > 0)
    hipLaunchKernelGGL(k_cnt_pairs, dim3(n_items), dim3(64), 0, s, n_items, v.n_rb, v.slot, v.slotY, ig, ih, listC, cntC,
                       actY, mC, mY, a0, a1, b0, b1, tri, out);
}

void launch_cnt_dot(size_t n, const int* a, const int* b, unsigned long long* dot, unsigned long long* sumb,
                    hipStream_t s) {
  unsigned int g = cgrid(n, 256);
  if (g > 1024) g = 1024;
  if (n) hipLaunchKernelGGL(k_cnt_dot, dim3(g), dim3(256), 0, s, n, a, b, dot, sumb);
}

}  // namespace sscf
