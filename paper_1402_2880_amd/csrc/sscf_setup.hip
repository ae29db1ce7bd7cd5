// Set-up kernels of the sparse SCF for gfx950 (MI355X, wave64): the steps that run once
// before the SCF loop.
//
// Paper: A. Scemama, N. Renon, M. Rapacioli, "A Sparse SCF algorithm and its
// parallel implementation: Application to DFTB", arXiv:1402.2880.
//
// Section 3.2: the atom neighbour map (k_tile_bbox, k_atom_nbr, k_row_scan), the MO-group
// neighbour map (k_group_nbr) and the constrained k-means that defines the groups (k_km_*).
// Section 3.3: the per-fragment initial guess
// (k_fragment_guess).  Squared distances are rounded operation by operation so that
// decisions taken on them (a neighbour cut, a nearest mean) are the ones of the plain IEEE
// expression.
#include "sscf_internal.h"

#include <math.h>

#include <algorithm>

namespace sscf {

// ---------------------------------------------------------------------------------------
// Set-up on the GPU (sections 3.2 and 3.3)
// ---------------------------------------------------------------------------------------

// (dx*dx + dy*dy) + dz*dz with every product and sum rounded on its own: contraction into
// fused multiply-adds is switched off here, so the result is the same double as the plain
// IEEE expression evaluated left to right on any machine.
__device__ __forceinline__ double sq_norm_rn(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

// Groups g and h are neighbours when an atom of g and an atom of h are closer than r_nbr.
// Workgroup g walks its atoms against all atoms; every hit stores 1 (no ordering needed).
__global__ void __launch_bounds__(256) k_group_nbr(int n_atoms, int G, const double* __restrict__ xyz,
                                                   const int* __restrict__ atom_group, const int* __restrict__ ga_ptr,
                                                   const int* __restrict__ ga, double r2, uint8_t* __restrict__ gnbr) {
  const int g = blockIdx.x;
  if (threadIdx.x == 0) gnbr[(size_t)g * G + g] = 1;
  const int n_g = ga_ptr[g + 1] - ga_ptr[g];
  for (size_t e = threadIdx.x; e < (size_t)n_g * n_atoms; e += blockDim.x) {
    const int a = ga[ga_ptr[g] + (int)(e / n_atoms)], b = (int)(e % n_atoms);
    const double dx = xyz[3 * a] - xyz[3 * b], dy = xyz[3 * a + 1] - xyz[3 * b + 1], dz = xyz[3 * a + 2] - xyz[3 * b + 2];
    const double d2 = sq_norm_rn(dx, dy, dz);
    if (d2 < r2) gnbr[(size_t)g * G + atom_group[b]] = 1;
  }
}

void launch_group_nbr(int n_atoms, int G, const double* xyz, const int* atom_group, const int* ga_ptr, const int* ga,
                      double r_nbr, uint8_t* gnbr, hipStream_t s) {
  hipLaunchKernelGGL(k_group_nbr, dim3(G), dim3(256), 0, s, n_atoms, G, xyz, atom_group, ga_ptr, ga, r_nbr * r_nbr,
                     gnbr);
}

// Initial guess of one fragment (section 3.3): H c = lambda S c on the fragment's own AOs,
// one thread per fragment (n <= GUESS_MAXN).  S = L L^T (Cholesky), A = L^-1 H L^-T, cyclic
// Jacobi on A with the 2 x 2 symmetric Schur rotation of each off-diagonal pair until the
// off-diagonal part is negligible, c = L^-T y; eigenpairs sorted by increasing lambda (stable),
// each vector's first entry within a relative 1e-10 of its largest |c| made positive (exactly
// equal entries of symmetric molecules would otherwise be decided by rounding).  out: n x n, column j =
// MO j, at frag_coff[f]; lam: n values at frag_aoff[f].  err |= 1: S not positive definite.
__global__ void __launch_bounds__(64) k_fragment_guess(int n_frag, const int* __restrict__ frag_atom0,
                                                       const int64_t* __restrict__ ao_off,
                                                       const int64_t* __restrict__ blk_rowptr,
                                                       const int* __restrict__ blk_col, const int64_t* __restrict__ blk_off,
                                                       const int* __restrict__ atom_nao, const double* __restrict__ Sv,
                                                       const double* __restrict__ Hv, const int64_t* __restrict__ frag_coff,
                                                       double* __restrict__ out, double* __restrict__ lam,
                                                       int* __restrict__ err) {
  constexpr int N = GUESS_MAXN;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_frag) return;
  const int a0 = frag_atom0[f], a1 = frag_atom0[f + 1];
  const int64_t lo = ao_off[a0];
  const int n = (int)(ao_off[a1] - lo);
  double S[N][N], A[N][N], V[N][N], L[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) { S[i][j] = 0.0; A[i][j] = 0.0; L[i][j] = 0.0; V[i][j] = (i == j) ? 1.0 : 0.0; }
  for (int a = a0; a < a1; ++a)
    for (int64_t k = blk_rowptr[a]; k < blk_rowptr[a + 1]; ++k) {
      const int b = blk_col[k];
      if (b < a0 || b >= a1) continue;
      const int na = atom_nao[a], nb = atom_nao[b];
      const int ra = (int)(ao_off[a] - lo), rb = (int)(ao_off[b] - lo);
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          S[ra + i][rb + j] = Sv[blk_off[k] + i * nb + j];
          A[ra + i][rb + j] = Hv[blk_off[k] + i * nb + j];
        }
    }
  // Cholesky S = L L^T
  for (int j = 0; j < n; ++j) {
    double d = S[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) { atomicOr(err, 1); return; }
    L[j][j] = sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = S[i][j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  // A <- L^-1 H (rows), then A <- A L^-T (columns); S is reused as scratch
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double v = A[i][c];
      for (int k = 0; k < i; ++k) v -= L[i][k] * S[k][c];
      S[i][c] = v / L[i][i];
    }
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double v = S[r][i];
      for (int k = 0; k < i; ++k) v -= L[i][k] * A[r][k];
      A[r][i] = v / L[i][i];
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) A[i][j] = A[j][i] = 0.5 * (A[i][j] + A[j][i]);
  // cyclic Jacobi
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < n; ++i) {
      dia += A[i][i] * A[i][i];
      for (int j = i + 1; j < n; ++j) off += A[i][j] * A[i][j];
    }
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  // order by increasing eigenvalue (stable)
  int ord[N];
  for (int i = 0; i < n; ++i) ord[i] = i;
  for (int i = 1; i < n; ++i) {
    const int o = ord[i];
    int j = i - 1;
    while (j >= 0 && A[ord[j]][ord[j]] > A[o][o]) { ord[j + 1] = ord[j]; --j; }
    ord[j + 1] = o;
  }
  double* C = out + frag_coff[f];
  for (int jj = 0; jj < n; ++jj) {
    const int j = ord[jj];
    double cv[N];
    for (int i = n - 1; i >= 0; --i) {        // c = L^-T y
      double v = V[i][j];
      for (int k = i + 1; k < n; ++k) v -= L[k][i] * cv[k];
      cv[i] = v / L[i][i];
    }
    double cm = 0.0;
    for (int i = 0; i < n; ++i) cm = fmax(cm, fabs(cv[i]));
    int km = 0;
    while (km < n - 1 && fabs(cv[km]) < cm * (1.0 - 1e-10)) ++km;
    const double sg = (cv[km] < 0.0) ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) C[i * n + jj] = sg * cv[i];
    lam[lo + jj] = A[j][j];
  }
}

void launch_fragment_guess(int n_frag, const int* frag_atom0, const int64_t* ao_off, const int64_t* blk_rowptr,
                           const int* blk_col, const int64_t* blk_off, const int* atom_nao, const double* S,
                           const double* H, const int64_t* frag_coff, double* out, double* lam, int* err,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_fragment_guess, dim3((n_frag + 63) / 64), dim3(64), 0, s, n_frag, frag_atom0, ao_off,
                     blk_rowptr, blk_col, blk_off, atom_nao, S, H, frag_coff, out, lam, err);
}

}  // namespace sscf


namespace sscf {

// ---------------------------------------------------------------------------------------
// Constrained k-means of section 3.2.  Every point is linked to one mean and no mean holds
// more than n_link points.  The attribution is the stable matching reached when points
// propose to means in order of increasing squared distance (ties: lower mean index) and
// every mean keeps its n_link closest candidates (ties: lower point index): no point would
// rather be at a mean that has room or holds a point farther from it.  The matching does
// not depend on the order in which points are visited, so the rounds below are fully
// parallel: all free points propose at once (k_km_propose), every mean merges its kept
// points with its new proposers and keeps the best n_link (k_km_accept); a point turned
// away proposes to its next mean in the following round.  Then every mean moves to the
// centroid of its points, summed in point order (k_km_centroid), and the summed
// displacement of the means decides the next iteration (k_km_disp).
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ double km_d2(const double* __restrict__ p, double cx, double cy, double cz) {
  return sq_norm_rn(p[0] - cx, p[1] - cy, p[2] - cz);
}

// (key, id) pairs in LDS, n2 a power of two, sorted ascending by key then id; all threads of
// the workgroup take part (blockDim.x threads), the last barrier is inside.
__device__ __forceinline__ void km_bitonic(double* key, int* id, int n2) {
  for (int size = 2; size <= n2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (n2 >> 1); t += blockDim.x) {
        const int i = (t / stride) * 2 * stride + (t % stride), j = i + stride;
        const bool up = (i & size) == 0;
        const bool gt = key[i] > key[j] || (key[i] == key[j] && id[i] > id[j]);
        if (gt == up) {
          const double tk = key[i]; key[i] = key[j]; key[j] = tk;
          const int ti = id[i]; id[i] = id[j]; id[j] = ti;
        }
      }
      __syncthreads();
    }
}

// rank[p * m + k] = index of the k-th nearest mean of point p; workgroup p sorts its m2
// (power of two >= m) candidates in LDS (dynamic: m2 doubles, then m2 ints).
__global__ void __launch_bounds__(256) k_km_rank(int m, int m2, const double* __restrict__ pts,
                                                 const double* __restrict__ means, int* __restrict__ rank) {
  extern __shared__ double km_rank_lds[];
  double* key = km_rank_lds;
  int* id = reinterpret_cast<int*>(km_rank_lds + m2);
  const int p = blockIdx.x;
  const double px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
  for (int k = threadIdx.x; k < m2; k += blockDim.x) {
    key[k] = k < m ? sq_norm_rn(px - means[3 * k], py - means[3 * k + 1], pz - means[3 * k + 2]) : INFINITY;
    id[k] = k < m ? k : 0x7fffffff;
  }
  __syncthreads();
  km_bitonic(key, id, m2);
  for (int k = threadIdx.x; k < m; k += blockDim.x) rank[(size_t)p * m + k] = id[k];
}

// every point free, every mean empty
__global__ void k_km_reset(int n, int m, int* __restrict__ assign, int* __restrict__ next, int* __restrict__ n_held,
                           int* __restrict__ pcnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) { assign[i] = -1; next[i] = 0; }
  if (i < m) { n_held[i] = 0; pcnt[i] = 0; }
}

// prop[p] = mean that free point p proposes to this round (-1: p is placed); pcnt[c] counts
// the proposals to mean c and plist holds the first KM_PCAP of them (in no particular order);
// clears the round's count of turned-away points
__global__ void k_km_propose(int n, int m, const int* __restrict__ rank, const int* __restrict__ assign,
                             const int* __restrict__ next, int* __restrict__ prop, int* __restrict__ pcnt,
                             int* __restrict__ plist, int* __restrict__ n_free) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) *n_free = 0;
  if (p >= n) return;
  const int c = (assign[p] < 0 && next[p] < m) ? rank[(size_t)p * m + next[p]] : -1;
  prop[p] = c;
  if (c >= 0) {
    const int slot = atomicAdd(&pcnt[c], 1);
    if (slot < KM_PCAP) plist[(size_t)c * KM_PCAP + slot] = p;
  }
}

// Workgroup c: candidates are the points it holds and the points proposing to it.  With at
// most KM_PCAP proposals they come from the mean's own list; otherwise the proposals are
// scanned in chunks of KM_SLOTS - n_link points so that the candidates always fit in LDS.
// Whenever there are more than n_link candidates they are sorted and the ones past n_link are
// turned away at once (a held point loses its place, a proposer moves on to its next mean).
// The sort by (squared distance, index) makes the arrival order of the proposals irrelevant.
// A point is a candidate of exactly one mean in a round, so its assign/next entries are
// written by one workgroup only.  A mean without proposals keeps what it holds.
__global__ void __launch_bounds__(256) k_km_accept(int n, int n_link, const double* __restrict__ pts,
                                                   const double* __restrict__ means, const int* __restrict__ prop,
                                                   int* __restrict__ pcnt, const int* __restrict__ plist,
                                                   int* __restrict__ assign, int* __restrict__ next,
                                                   int* __restrict__ held, int* __restrict__ n_held,
                                                   int* __restrict__ n_free) {
  __shared__ double key[KM_SLOTS];
  __shared__ int id[KM_SLOTS];
  __shared__ int cnt;
  const int c = blockIdx.x;
  const int np = pcnt[c];
  if (np == 0) return;
  const double cx = means[3 * c], cy = means[3 * c + 1], cz = means[3 * c + 2];
  int kept = n_held[c];
  for (int t = threadIdx.x; t < kept; t += blockDim.x) {
    const int p = held[(size_t)c * n_link + t];
    id[t] = p;
    key[t] = km_d2(pts + 3 * p, cx, cy, cz);
  }
  // candidates [0, total) in LDS: keep the best n_link, turn the rest away
  auto settle = [&](int total) -> int {
    if (total <= n_link) return total;
    int n2 = 1;
    while (n2 < total) n2 <<= 1;                  // n2 <= KM_SLOTS
    for (int s = total + threadIdx.x; s < n2; s += blockDim.x) { key[s] = INFINITY; id[s] = 0x7fffffff; }
    __syncthreads();
    km_bitonic(key, id, n2);
    for (int s = n_link + threadIdx.x; s < total; s += blockDim.x) {
      const int p = id[s];
      if (assign[p] == c) assign[p] = -1;
      next[p] += 1;
      atomicAdd(n_free, 1);
    }
    return n_link;
  };
  if (np <= KM_PCAP) {
    if (threadIdx.x == 0) cnt = kept;
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
      const int p = plist[(size_t)c * KM_PCAP + i];
      const int s = atomicAdd(&cnt, 1);           // s < n_link + KM_PCAP <= KM_SLOTS
      id[s] = p;
      key[s] = km_d2(pts + 3 * p, cx, cy, cz);
    }
    __syncthreads();
    kept = settle(cnt);
    __syncthreads();
  } else {
    const int chunk = KM_SLOTS - n_link;
    for (int base = 0; base < n; base += chunk) {
      if (threadIdx.x == 0) cnt = kept;
      __syncthreads();
      const int end = min(n, base + chunk);
      for (int p = base + threadIdx.x; p < end; p += blockDim.x)
        if (prop[p] == c) {
          const int s = atomicAdd(&cnt, 1);       // s < kept + chunk <= KM_SLOTS
          id[s] = p;
          key[s] = km_d2(pts + 3 * p, cx, cy, cz);
        }
      __syncthreads();
      kept = settle(cnt);
      __syncthreads();
    }
  }
  for (int s = threadIdx.x; s < kept; s += blockDim.x) {
    const int p = id[s];
    held[(size_t)c * n_link + s] = p;
    assign[p] = c;
  }
  if (threadIdx.x == 0) { n_held[c] = kept; pcnt[c] = 0; }
}

// workgroup c: centroid of mean c's points, coordinates summed in point order and divided by
// the count (a mean without points stays where it is).  The points are first listed in
// ascending order (ballot compaction, waves in order), then summed by one thread.
__global__ void __launch_bounds__(256) k_km_centroid(int n, int m, const double* __restrict__ pts,
                                                     const int* __restrict__ assign,
                                                     const double* __restrict__ means, double* __restrict__ out) {
  __shared__ int idx[KM_MAX_LINK];
  __shared__ int wcnt[4];
  const int c = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int k = 0;                                          // points listed so far (same in every thread)
  for (int base = 0; base < n; base += 256) {
    const int p = base + (int)threadIdx.x;
    const bool f = p < n && assign[p] == c;
    const unsigned long long bal = __ballot(f);
    if (lane == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int off = k;
    for (int v = 0; v < w; ++v) off += wcnt[v];
    if (f) {
      const int slot = off + __popcll(bal & ((1ull << lane) - 1ull));
      if (slot < KM_MAX_LINK) idx[slot] = p;          // a mean holds at most n_link <= KM_MAX_LINK points
    }
    k += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  k = min(k, KM_MAX_LINK);
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int i = 0; i < k; ++i) {
    const int p = idx[i];
    sx += pts[3 * p];
    sy += pts[3 * p + 1];
    sz += pts[3 * p + 2];
  }
  if (k == 0) {
    out[3 * c] = means[3 * c]; out[3 * c + 1] = means[3 * c + 1]; out[3 * c + 2] = means[3 * c + 2];
  } else {
    const double dk = (double)k;
    out[3 * c] = sx / dk; out[3 * c + 1] = sy / dk; out[3 * c + 2] = sz / dk;
  }
}

// sum over the means, in mean order, of |new - old| (one thread)
__global__ void k_km_disp(int m, const double* __restrict__ old_means, const double* __restrict__ new_means,
                          double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int c = 0; c < m; ++c)
    s += __dsqrt_rn(sq_norm_rn(new_means[3 * c] - old_means[3 * c], new_means[3 * c + 1] - old_means[3 * c + 1],
                               new_means[3 * c + 2] - old_means[3 * c + 2]));
  *out = s;
}

void launch_km_rank(int n, int m, const double* pts, const double* means, int* rank, hipStream_t s) {
  int m2 = 1;
  while (m2 < m) m2 <<= 1;
  hipLaunchKernelGGL(k_km_rank, dim3(n), dim3(256), (size_t)m2 * (sizeof(double) + sizeof(int)), s, m, m2, pts,
                     means, rank);
}
void launch_km_reset(int n, int m, int* assign, int* next, int* n_held, int* pcnt, hipStream_t s) {
  const int t = std::max(n, m);
  hipLaunchKernelGGL(k_km_reset, dim3((t + 255) / 256), dim3(256), 0, s, n, m, assign, next, n_held, pcnt);
}
void launch_km_round(int n, int m, int n_link, const double* pts, const double* means, const int* rank, int* assign,
                     int* next, int* prop, int* pcnt, int* plist, int* held, int* n_held, int* n_free, hipStream_t s) {
  hipLaunchKernelGGL(k_km_propose, dim3((n + 255) / 256), dim3(256), 0, s, n, m, rank, assign, next, prop, pcnt,
                     plist, n_free);
  hipLaunchKernelGGL(k_km_accept, dim3(m), dim3(256), 0, s, n, n_link, pts, means, prop, pcnt, plist, assign, next,
                     held, n_held, n_free);
}
void launch_km_move(int n, int m, const double* pts, const int* assign, const double* means, double* out,
                    double* disp, hipStream_t s) {
  hipLaunchKernelGGL(k_km_centroid, dim3(m), dim3(256), 0, s, n, m, pts, assign, means, out);
  hipLaunchKernelGGL(k_km_disp, dim3(1), dim3(64), 0, s, m, means, out, disp);
}

}  // namespace sscf

namespace sscf {

// ---------------------------------------------------------------------------------------
// Atom neighbour map of section 3.2: atoms a and b are neighbours when some S or H element
// between their AOs can be nonzero, which for two-centre elements with a radial cut-off means
// |r_a - r_b|^2 < cutoff^2 (every atom is its own neighbour).  Output: CSR rows in atom order,
// columns ascending.  The atoms are cut into tiles of 64 consecutive atoms; the wave of tile A
// (one lane per atom a) walks every tile B whose bounding box can come within the cut-off and
// tests the 64 atoms of B one after the other, so each lane meets its columns in ascending
// order.  The bounding-box test only skips a tile when its gap exceeds the cut-off by a
// relative 1e-9, far more than the rounding of the gap, so no neighbour is ever skipped; the
// decision on each pair is taken on the rounded squared distance alone.
// ---------------------------------------------------------------------------------------

constexpr int NB_TILE = 64;
static_assert(NB_TILE == NB_TILE_ATOMS, "tile size of the atom neighbour map");

// lo/hi corners of each tile's atoms (exact: min and max round nothing)
__global__ void __launch_bounds__(64) k_tile_bbox(int n, const double* __restrict__ xyz, double* __restrict__ box) {
  const int t = blockIdx.x, a = t * NB_TILE + threadIdx.x;
  const bool in = a < n;
  double lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = in ? xyz[3 * a + d] : INFINITY;
    hi[d] = in ? xyz[3 * a + d] : -INFINITY;
  }
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], __shfl_xor(lo[d], o));
      hi[d] = fmax(hi[d], __shfl_xor(hi[d], o));
    }
  if (threadIdx.x == 0)
#pragma unroll
    for (int d = 0; d < 3; ++d) { box[6 * t + d] = lo[d]; box[6 * t + 3 + d] = hi[d]; }
}

// fill = 0: cnt[a] = number of neighbours of a.  fill = 1: col[rowptr[a] ..] = neighbours.
__global__ void __launch_bounds__(64) k_atom_nbr(int n, const double* __restrict__ xyz, const double* __restrict__ box,
                                                 double c2, double c2_skip, int fill, int* __restrict__ cnt,
                                                 const int64_t* __restrict__ rowptr, int* __restrict__ col) {
  __shared__ double bx[NB_TILE * 3];
  const int ta = blockIdx.x, n_tiles = (n + NB_TILE - 1) / NB_TILE;
  const int a = ta * NB_TILE + threadIdx.x;
  const bool in = a < n;
  const double ax = in ? xyz[3 * a] : 0.0, ay = in ? xyz[3 * a + 1] : 0.0, az = in ? xyz[3 * a + 2] : 0.0;
  const double* A = box + 6 * ta;
  int k = 0;
  int64_t w = (fill && in) ? rowptr[a] : 0;
  for (int tb = 0; tb < n_tiles; ++tb) {
    const double* B = box + 6 * tb;
    const double gx = fmax(0.0, fmax(B[0] - A[3], A[0] - B[3]));
    const double gy = fmax(0.0, fmax(B[1] - A[4], A[1] - B[4]));
    const double gz = fmax(0.0, fmax(B[2] - A[5], A[2] - B[5]));
    if (sq_norm_rn(gx, gy, gz) > c2_skip) continue;          // wave-uniform
    const int b0 = tb * NB_TILE, nb = min(NB_TILE, n - b0);
    __syncthreads();
    if ((int)threadIdx.x < nb) {
      bx[3 * threadIdx.x] = xyz[3 * (b0 + threadIdx.x)];
      bx[3 * threadIdx.x + 1] = xyz[3 * (b0 + threadIdx.x) + 1];
      bx[3 * threadIdx.x + 2] = xyz[3 * (b0 + threadIdx.x) + 2];
    }
    __syncthreads();
    if (!in) continue;
    for (int j = 0; j < nb; ++j) {
      const bool hit = sq_norm_rn(ax - bx[3 * j], ay - bx[3 * j + 1], az - bx[3 * j + 2]) < c2;
      if (hit) {
        if (fill) col[w++] = b0 + j;
        else ++k;
      }
    }
  }
  if (!fill && in) cnt[a] = k;
}

// rowptr[0] = 0, rowptr[a + 1] = rowptr[a] + cnt[a] (one workgroup of 1024 threads; thread t
// sums a contiguous chunk, the chunk sums are scanned in LDS, then every chunk is written)
__global__ void __launch_bounds__(1024) k_row_scan(int n, const int* __restrict__ cnt, int64_t* __restrict__ rowptr) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x, per = (n + 1023) / 1024;
  const int i0 = min(n, t * per), i1 = min(n, i0 + per);
  int64_t s = 0;
  for (int i = i0; i < i1; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;                                // exclusive prefix of chunk t
  if (t == 0) rowptr[0] = 0;
  for (int i = i0; i < i1; ++i) {
    run += cnt[i];
    rowptr[i + 1] = run;
  }
}

// flag = 1 when a coordinate is not finite or exceeds 1e100 in magnitude (flag cleared by the caller)
__global__ void k_check_coords(int64_t n, const double* __restrict__ x, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!(fabs(x[i]) <= 1e100)) *flag = 1;
}
void launch_check_coords(int64_t n, const double* x, int* flag, hipStream_t s) {
  const int64_t g = (n + 255) / 256;
  if (n) hipLaunchKernelGGL(k_check_coords, dim3((unsigned int)(g < 1024 ? g : 1024)), dim3(256), 0, s, n, x, flag);
}

void launch_atom_nbr_count(int n, const double* xyz, double cutoff, double* box, int* cnt, int64_t* rowptr,
                           hipStream_t s) {
  const int nt = (n + NB_TILE - 1) / NB_TILE;
  const double c2 = cutoff * cutoff;
  hipLaunchKernelGGL(k_tile_bbox, dim3(nt), dim3(64), 0, s, n, xyz, box);
  hipLaunchKernelGGL(k_atom_nbr, dim3(nt), dim3(64), 0, s, n, xyz, box, c2, c2 * (1.0 + 1e-9), 0, cnt,
                     (const int64_t*)nullptr, (int*)nullptr);
  hipLaunchKernelGGL(k_row_scan, dim3(1), dim3(1024), 0, s, n, cnt, rowptr);
}
void launch_atom_nbr_fill(int n, const double* xyz, double cutoff, const double* box, const int64_t* rowptr, int* col,
                          hipStream_t s) {
  const int nt = (n + NB_TILE - 1) / NB_TILE;
  const double c2 = cutoff * cutoff;
  hipLaunchKernelGGL(k_atom_nbr, dim3(nt), dim3(64), 0, s, n, xyz, box, c2, c2 * (1.0 + 1e-9), 1, (int*)nullptr,
                     rowptr, col);
}

}  // namespace sscf
