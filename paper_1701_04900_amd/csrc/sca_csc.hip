// Sparse path of libsca: A given in CSR is converted once to a library-owned CSC
// (rows ascending inside every column).  A round reads, per drawn coordinate, the nonzeros
// of its column (value + row index) and gathers r from L2.  The residual fold is a
// scatter-add into r, done without global atomics and bitwise reproducibly: rows are cut
// into bins of R = 2^bin_log rows; the gradient kernel counts, per workgroup and bin, the
// nonzeros of its moved columns; a scan turns the counts into slots; a scatter pass writes
// (row within bin, a_ij * dx_j) entries into the slots; one workgroup per bin adds its
// entries into fixed-point cells in LDS (exact at 2^-72, so the order of the additions
// does not matter) and adds the cells to r in one rounding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "sca_internal.h"

using namespace sca;

namespace {


// ------------------------------------------------------------------ CSR -> CSC
__global__ void k_count_cols(const int32_t* __restrict__ colidx, long long nnz, int n,
                             int* __restrict__ colcnt, int* __restrict__ bad) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nnz;
       k += (long long)gridDim.x * blockDim.x) {
    const int j = colidx[k];
    if (j < 0 || j >= n) {
      atomicOr(bad, 1);
    } else {
      atomicAdd(&colcnt[j], 1);
    }
  }
}

// One wave per CSR row: every entry goes to the next free slot of its column (slot
// order is arbitrary; the per-column sort below fixes it).
template <typename T>
__global__ void k_scatter_cols(const long long* __restrict__ rowptr,
                               const int32_t* __restrict__ colidx, const T* __restrict__ vals,
                               int m, const long long* __restrict__ colptr,
                               int* __restrict__ cursor, int* __restrict__ tmp_row,
                               long long* __restrict__ tmp_src) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * (blockDim.x >> 6);
  for (int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < m; i += nw) {
    for (long long k = rowptr[i] + lane; k < rowptr[i + 1]; k += 64) {
      const int j = colidx[k];
      const long long pos = colptr[j] + atomicAdd(&cursor[j], 1);
      tmp_row[pos] = i;
      tmp_src[pos] = k;
    }
  }
}

// One wave per column: rank of each entry by (row, source position) = its final slot.
template <typename T>
__global__ void k_sort_cols(const long long* __restrict__ colptr, int n,
                            const int* __restrict__ tmp_row, const long long* __restrict__ tmp_src,
                            const T* __restrict__ vals, int* __restrict__ rowidx,
                            T* __restrict__ cvals, int* __restrict__ dup) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * (blockDim.x >> 6);
  for (int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); j < n; j += nw) {
    const long long b = colptr[j], e = colptr[j + 1];
    for (long long p = b + lane; p < e; p += 64) {
      const int rp = tmp_row[p];
      const long long sp = tmp_src[p];
      long long rank = 0;
      for (long long q = b; q < e; ++q) {
        const int rq = tmp_row[q];
        if (rq < rp || (rq == rp && tmp_src[q] < sp)) ++rank;
        if (rq == rp && q != p) atomicOr(dup, 1);
      }
      rowidx[b + rank] = rp;
      cvals[b + rank] = vals[sp];
    }
  }
}

template <typename T>
__global__ void k_colnorm2_csc(const long long* __restrict__ colptr, const T* __restrict__ v,
                               int n, double* __restrict__ cn2) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (long long k = colptr[j]; k < colptr[j + 1]; ++k) {
      const double a = (double)v[k];
      s += a * a;
    }
    cn2[j] = s;
  }
}

// ------------------------------------------------------------------ round kernels
constexpr int kBinMaxLog = 10;     // bins of at most 1024 rows: 32 KiB of limb cells
constexpr int kBinMinLog = 6;
constexpr int kMaxBins = 8192;     // histogram of a workgroup: 32 KiB of LDS
constexpr int kCscThreads = 1024;  // 64 groups of 16 lanes; one listed column per group
constexpr int kBinGridMax = 4096;  // workgroups of the counting kernels (scan: 16 per thread)

// Exclusive scan over a block of NW waves; 'sh' needs NW + 1 ints.  Contains __syncthreads.
template <int NW>
__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < NW; ++w) {
      const int t = sh[w];
      sh[w] = run;
      run += t;
    }
    sh[NW] = run;
  }
  __syncthreads();
  const int res = sh[wave] + inc - v;
  *total = sh[NW];
  __syncthreads();
  return res;
}

// Sum of 16 lanes (xor butterfly inside each aligned group of 16; every lane of the group
// ends with the same, bitwise identical value).
template <typename Acc> __device__ __forceinline__ Acc sum16(Acc s) {
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
  return s;
}

template <typename T, typename TR, typename Acc>
__device__ __forceinline__ Acc csc_col_dot(const long long* __restrict__ colptr,
                                           const int* __restrict__ rowidx,
                                           const T* __restrict__ v, const TR* __restrict__ r,
                                           int j, int sub) {
  Acc s = (Acc)0;
  const long long b = colptr[j], e = colptr[j + 1];
  for (long long k = b + sub; k < e; k += 16) s += (Acc)v[k] * (Acc)r[rowidx[k]];
  return sum16(s);
}

// Work mapping shared by the counting, gradient and scatter kernels: workgroup w takes the
// contiguous chunk [c0, c1) of the S listed items (ceil(S / grid) each); inside it, groups
// of 16 lanes take items c0 + group, c0 + group + groups, ...
__device__ __forceinline__ void wg_chunk(int S, int* c0, int* c1) {
  const long long per = ((long long)S + gridDim.x - 1) / gridDim.x;
  const long long a = min((long long)S, (long long)blockIdx.x * per);
  *c0 = (int)a;
  *c1 = (int)min((long long)S, a + per);
}

__device__ __forceinline__ void flush_counts(const int* hist, int nb, int moved, int* s_moved,
                                             int* __restrict__ cnt, int* __restrict__ moved_wg) {
  const int wm = (int)wave_sum_i64((long long)moved);
  if ((threadIdx.x & 63) == 0) s_moved[threadIdx.x >> 6] = wm;
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) cnt[(size_t)blockIdx.x * nb + i] = hist[i];
  if (threadIdx.x == 0 && moved_wg) {
    int tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += s_moved[w];
    moved_wg[blockIdx.x] = tot;
  }
}

// Best response and step of drawn coordinate t (column j) from its dot product a_j^T r;
// every lane of the group computes the same d, lane 0 stores.
// The same from x_j and ||a_j||^2 already loaded.
template <typename T>
__device__ __forceinline__ T csc_step_v(T dot, T xj, double cn2j, int j, int t, int sub, T gamma,
                                        T* __restrict__ x, T* __restrict__ dx_sel,
                                        const BRParams& bp) {
  T g = dot - (T)bp.c2 * xj;
  if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
  const T q = (T)(cn2j + bp.tau);
  const T xh = soft_clip<T>(xj - g / q, (T)bp.lam_eta / q, (T)bp.beta);
  const T d = gamma * (xh - xj);
  if (sub == 0) {
    x[j] = xj + d;
    dx_sel[t] = d;
  }
  return d;
}

template <typename T>
__device__ __forceinline__ T csc_step(T dot, int j, int t, int sub, T gamma, T* __restrict__ x,
                                      const double* __restrict__ cn2, T* __restrict__ dx_sel,
                                      const BRParams& bp) {
  return csc_step_v<T>(dot, x[j], cn2[j], j, t, sub, gamma, x, dx_sel, bp);
}

// S.2 + S.4 on sparse columns with r gathered from memory (used when the panel kernel
// below does not apply): 16 lanes per drawn coordinate; the first 16*U nonzeros are loaded
// at once, longer columns continue in a loop.  The moved columns' nonzeros are counted per
// row bin in LDS; the counts go to cnt[blockIdx.x][bin], the number of moved columns to
// moved_wg[blockIdx.x].
template <typename T, int U>
__global__ void __launch_bounds__(kCscThreads)
k_grad_br_csc(const long long* __restrict__ colptr, const int* __restrict__ rowidx,
              const T* __restrict__ v, const T* __restrict__ r, T* __restrict__ x,
              const double* __restrict__ cn2, const int* __restrict__ sel_cols,
              const RoundState* __restrict__ st, T* __restrict__ dx_sel, BRParams bp,
              int bin_log, int nb, int* __restrict__ cnt, int* __restrict__ moved_wg) {
  extern __shared__ int hist[];
  __shared__ int s_moved[kCscThreads / 64];
  for (int i = threadIdx.x; i < nb; i += kCscThreads) hist[i] = 0;
  __syncthreads();
  const int sub = threadIdx.x & 15;
  const T gamma = (T)st->gamma_cur;
  int c0, c1;
  wg_chunk(st->S_cnt, &c0, &c1);
  int moved = 0;
  for (int t = c0 + (int)(threadIdx.x >> 4); t < c1; t += kCscThreads / 16) {
    const int j = sel_cols[t];
    const long long b = colptr[j], e = colptr[j + 1];
    int ri[U];
    T vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long k = b + sub + 16 * u;
      ri[u] = k < e ? rowidx[k] : -1;
      vv[u] = k < e ? v[k] : (T)0;
    }
    T s = (T)0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ri[u] >= 0) s += vv[u] * r[ri[u]];
    for (long long k = b + sub + 16 * U; k < e; k += 16) s += v[k] * r[rowidx[k]];
    const T d = csc_step<T>(sum16(s), j, t, sub, gamma, x, cn2, dx_sel, bp);
    if (d != (T)0) {
      moved += sub == 0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ri[u] >= 0) atomicAdd(&hist[ri[u] >> bin_log], 1);
      for (long long k = b + sub + 16 * U; k < e; k += 16)
        atomicAdd(&hist[rowidx[k] >> bin_log], 1);
    }
  }
  flush_counts(hist, nb, moved, s_moved, cnt, moved_wg);
}

// S.2 + S.4 with r staged in LDS: one 1024-thread workgroup per CU walks the rows in
// equal panels of at most 128 KiB; for each panel it copies r's panel into LDS (loads unrolled in batches
// of 16 per thread and issued together with the column loads), then every group of 16
// lanes advances a cursor through each of its columns (up to CPG per pass) over the
// nonzeros whose rows fall in the panel (rows ascend inside a column, so they form a prefix
// of each 32-entry window), with r read from LDS.  Each lane keeps its partial sums across
// panels; the 16 partial sums of a column are added at the end in a fixed order.  Then the
// best response, the step and the bin counts of the moved columns as in the kernel above.
constexpr int kPanelBytes = 131072;
constexpr int kPanelMaxBins = 2048;
constexpr int kPanelThreads = 1024;
constexpr int kPanelGroups = kPanelThreads / 16;
constexpr int kPanelBatch = 16;
template <typename T, int CPG>
__global__ void __launch_bounds__(kPanelThreads)
k_grad_br_cscp(const long long* __restrict__ colptr, const int* __restrict__ rowidx,
               const T* __restrict__ v, const T* __restrict__ r, T* __restrict__ x,
               const double* __restrict__ cn2, const int* __restrict__ sel_cols,
               const RoundState* __restrict__ st, T* __restrict__ dx_sel, BRParams bp, int m,
               int bin_log, int nb, int* __restrict__ cnt, int* __restrict__ moved_wg) {
  constexpr int PR = kPanelBytes / (int)sizeof(T);
  __shared__ T s_r[PR];
  __shared__ int hist[kPanelMaxBins];
  __shared__ int s_moved[kPanelThreads / 64];
  for (int i = threadIdx.x; i < nb; i += kPanelThreads) hist[i] = 0;
  const int sub = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int gshift = 16 * ((threadIdx.x & 63) >> 4);
  const T gamma = (T)st->gamma_cur;
  int c0, c1;
  wg_chunk(st->S_cnt, &c0, &c1);
  // equal panels of at most PR rows (multiples of 64)
  const int NP = (m + PR - 1) / PR;
  const int PE = ((m + NP - 1) / NP + 63) / 64 * 64;
  int moved = 0;
  for (int pb = c0; pb < c1; pb += kPanelGroups * CPG) {
    int kc[CPG], ke[CPG], jj[CPG];
    T acc[CPG];
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      const int t = pb + grp + kPanelGroups * i;
      jj[i] = -1;
      kc[i] = ke[i] = 0;
      acc[i] = (T)0;
      if (t < c1) {
        jj[i] = sel_cols[t];
        kc[i] = (int)colptr[jj[i]];
        ke[i] = (int)colptr[jj[i] + 1];
      }
    }
    for (int P = 0; P < NP; ++P) {
      const int lo = P * PE, hi = min(m, lo + PE), len = hi - lo;
      // the next 32 entries of every column
      int rw[CPG][2];
      T vw[CPG][2];
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = kc[i] + sub + 16 * h;
          rw[i][h] = k < ke[i] ? rowidx[k] : INT_MAX;
          vw[i][h] = k < ke[i] ? v[k] : (T)0;
        }
      }
      // r's panel into LDS: a batch of loads per thread, then (after every wave has left
      // the previous panel) the stores
      for (int base = 0; base < len; base += kPanelThreads * kPanelBatch) {
        T tmp[kPanelBatch];
#pragma unroll
        for (int u = 0; u < kPanelBatch; ++u) {
          const int i = base + (int)threadIdx.x + u * kPanelThreads;
          tmp[u] = i < len ? r[lo + i] : (T)0;
        }
        if (base == 0) __syncthreads();
#pragma unroll
        for (int u = 0; u < kPanelBatch; ++u) {
          const int i = base + (int)threadIdx.x + u * kPanelThreads;
          if (i < len) s_r[i] = tmp[u];
        }
      }
      __syncthreads();
      // windows that lay wholly inside the panel continue with the next 32 entries; the
      // loads of all such columns are issued together
      bool more = true;
      while (more) {
        more = false;
#pragma unroll
        for (int i = 0; i < CPG; ++i) {
          int nin = 0;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const bool in = rw[i][h] < hi;
            if (in) acc[i] += vw[i][h] * s_r[rw[i][h] - lo];
            nin += __popcll((__ballot(in) >> gshift) & 0xffffull);
          }
          kc[i] += nin;
          const bool full = nin == 32;
          more |= full;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int k = kc[i] + sub + 16 * h;
            rw[i][h] = full && k < ke[i] ? rowidx[k] : INT_MAX;
            vw[i][h] = full && k < ke[i] ? v[k] : (T)0;
          }
        }
      }
    }
    // best responses: x_j and ||a_j||^2 of every column of the pass loaded together
    T xj[CPG];
    double qj[CPG];
    int kb[CPG];
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      xj[i] = jj[i] >= 0 ? x[jj[i]] : (T)0;
      qj[i] = jj[i] >= 0 ? cn2[jj[i]] : 0.0;
      kb[i] = jj[i] >= 0 ? (int)colptr[jj[i]] : 0;
    }
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      if (jj[i] < 0) continue;
      const int t = pb + grp + kPanelGroups * i;
      const T d = csc_step_v<T>(sum16(acc[i]), xj[i], qj[i], jj[i], t, sub, gamma, x, dx_sel, bp);
      if (d != (T)0)
        moved += sub == 0;
      else
        kb[i] = ke[i];  // not moved: no bin counts
    }
    // bin counts of the moved columns' nonzeros, 64 entries of every moved column per step
    // (four loads per lane for each column in flight together)
    for (int o = 0;; o += 64) {
      int rr[CPG][4];
#pragma unroll
      for (int i = 0; i < CPG; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = kb[i] + o + sub + 16 * u;
          rr[i][u] = rowidx[jj[i] >= 0 && k < ke[i] ? k : 0];
        }
      bool left = false;
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (jj[i] >= 0 && kb[i] + o + sub + 16 * u < ke[i])
            atomicAdd(&hist[rr[i][u] >> bin_log], 1);
        left |= jj[i] >= 0 && kb[i] + o + 64 < ke[i];
      }
      if (!left) break;
    }
    __syncthreads();  // the next pass refills the panels
  }
  __syncthreads();
  flush_counts(hist, nb, moved, s_moved, cnt, moved_wg);
}

// Panel-split gradient.  The rows are cut into NP <= kSplitMaxPanels panels of PE rows
// (PE <= kSplitPanelBytes / sizeof(T)); pofs[j * (NP + 1) + P] is the first entry of column
// j whose row lies in panel P (rows ascend inside a column), written once at create time.
constexpr int kSplitPanelBytes = 143360;  // 140 KiB of r per workgroup
constexpr int kSplitMaxPanels = 16;       // one partial per lane of a 16-lane group
constexpr int kSplitList = 2048;          // drawn columns listed in LDS at a time (in-kernel draw)

// pofs of every column: a binary search per inner panel boundary.
__global__ void __launch_bounds__(256)
k_panel_offsets(const long long* __restrict__ colptr, const int* __restrict__ rowidx, int n,
                int NP, int PE, int* __restrict__ pofs) {
  for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
    const int b = (int)colptr[j], e = (int)colptr[j + 1];
    int* o = pofs + (size_t)j * (NP + 1);
    o[0] = b;
    o[NP] = e;
    for (int P = 1; P < NP; ++P) {
      const int target = P * PE;
      int lo = b, hi = e;
      while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (rowidx[mid] < target)
          lo = mid + 1;
        else
          hi = mid;
      }
      o[P] = lo;
    }
  }
}

// Partial dot products a_j^T r over one panel (S.2 of Algorithm 1, first half).  Workgroup
// w takes panel P = w % NP, stages r's rows of that panel in LDS once, and walks chunk
// w / NP (of CPP equal chunks) of the drawn list: 16 lanes per drawn coordinate, CPG
// coordinates per group in flight, the panel's first 48 entries of each loaded at once
// (longer runs continue four loads at a time); the next pass's panel offsets and the list
// entries of the pass after it are loaded while the current one computes.  Every load is unconditional (an index past the
// run reads entry 0, whose value is not used), so no load waits for another's result
// except through a real dependence.  Lane sub adds the entries sub, sub + 16, ... in order;
// part[P * ldpart + t] = the 16 lane sums added by sum16.
// DRAW: the block draw (S.1) runs here instead of in k_select: every workgroup draws every
// block of round st->k (at most 32 per thread: the drawn flags and the first list position
// of each thread's blocks are kept in LDS), scans the drawn columns in block order and lists
// the columns of its chunk in LDS, kSplitList at a time; the workgroups of panel 0 also
// write their chunk to sel_out for the kernels that follow, and workgroup 0 writes the
// drawn count.  The round state is advanced after the fold (k_bin_scan).  Without DRAW the
// list is sel_cols, walked in the same pieces.
template <typename T, int CPG, bool DRAW>
__global__ void __launch_bounds__(1024)
k_dot_split(const int* __restrict__ pofs, const int* __restrict__ rowidx,
            const T* __restrict__ v, const T* __restrict__ r, const int* __restrict__ sel_cols,
            RoundState* __restrict__ st, int m, int NP, int PE, int CPP,
            T* __restrict__ part, long long ldpart, FusedSel fs, int* __restrict__ sel_out) {
  constexpr int PR = kSplitPanelBytes / (int)sizeof(T);
  constexpr int G = 1024 / 16;  // groups of 16 lanes
  constexpr int H = 3;          // 16-entry windows loaded at once per coordinate
  __shared__ T s_r[PR];
  __shared__ int s_list[DRAW ? kSplitList : 1];
  __shared__ uint32_t s_dmask[DRAW ? 1024 : 1];
  __shared__ int s_doff[DRAW ? 1024 : 1];
  __shared__ int s_scan[17];
  // the NP panels of one chunk run on one XCD: the cache lines their column runs share
  // (a column's entries cross panel boundaries inside a line) are fetched into one L2
  const int g = xcd_order((int)blockIdx.x, (int)gridDim.x);
  const int P = g % NP, c = g / NP;
  const int lo = P * PE, hi = min(m, lo + PE), len = max(0, hi - lo);
  // r's rows of the panel go straight into LDS (16-byte direct-to-LDS loads, lane l of a wave
  // at base + 16 l), all issued at once behind the first pass's panel offsets, with one wait
  // for both (against three rounds of register staging: gradient step 48.9 -> 47.3 us).  A
  // lane past the panel's last whole 16-byte group reads its first one (its slot lies below
  // the panel's capacity and is never read; the last round, which would reach past the
  // capacity, is issued only where it starts inside the panel), and the last partial group (m
  // not a multiple of its elements) is loaded after the wait by the lane that owns it.
  constexpr int VN = 16 / (int)sizeof(T);
  const int nfull = len / VN;  // whole 16-byte groups of the panel
  auto stage_r = [&]() {
    const int wbase = (int)threadIdx.x & ~63;
    constexpr int NRB = (PR + 1024 * VN - 1) / (1024 * VN);
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      const int q0 = rb * 1024 + wbase;  // first group of this wave's segment
      // every round but the last lies inside the panel's capacity: issued unconditionally
      if (rb + 1 < NRB || q0 * VN < len) {
        const int q = q0 + ((int)threadIdx.x & 63);
        __builtin_amdgcn_global_load_lds(
            (const void*)(r + lo + (size_t)(q < nfull ? q : 0) * VN),
            (__attribute__((address_space(3))) void*)(s_r + (size_t)q0 * VN), 16, 0, 0);
      }
    }
  };
  const int dper = (fs.nblocks + 1023) / 1024;  // <= 32 (host check)
  const int db0 = min(fs.nblocks, (int)threadIdx.x * dper);
  const int db1 = min(fs.nblocks, db0 + dper);
  int S;
  if (DRAW) {
    // this thread's blocks [db0, db1): block pointers loaded four blocks at a time (all
    // loads in flight before the draws that use them), drawn flags, drawn column count
    const long long k = st->k;
    int cnt = 0;
    uint32_t dm = 0;
    for (int i0 = db0; i0 < db1; i0 += 4) {
      int bv[5];
#pragma unroll
      for (int u = 0; u < 5; ++u) bv[u] = fs_blk_begin(fs, min(i0 + u, fs.nblocks));
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u;
        if (i < db1 && block_drawn((uint32_t)i, (uint64_t)k, fs.inst, fs.seed, fs.T)) {
          cnt += bv[u + 1] - bv[u];
          dm |= 1u << (i - db0);
        }
      }
    }
    s_dmask[threadIdx.x] = dm;
    s_doff[threadIdx.x] = block_exclusive_scan_1024(cnt, s_scan, &S);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->S_cnt = S;
    __syncthreads();  // s_doff of the next thread is read below
  } else {
    S = st->S_cnt;
  }
  S = __builtin_amdgcn_readfirstlane(S);  // uniform: the chunk bounds stay in scalar registers
  // the columns of list positions [p0, p1) into s_list (panel 0 also writes them to
  // sel_out).  Only threads whose drawn columns [s_doff[t], s_doff[t + 1]) meet [p0, p1)
  // have blocks to list; each wave lists its lanes' blocks together, one block at a time,
  // 64 positions per store.
  auto expand = [&](int p0, int p1) {
    const int lane = threadIdx.x & 63;
    uint32_t dm = s_dmask[threadIdx.x];
    int o = s_doff[threadIdx.x];
    const int oend = threadIdx.x + 1 < 1024 ? s_doff[threadIdx.x + 1] : S;
    if (oend <= p0 || o >= p1) dm = 0;
    for (;;) {
      int cb = 0, oo = 0, a = 0, b = 0;
      bool have = false;
      while (dm != 0 && o < p1) {  // this thread's next drawn block that meets [p0, p1)
        const int i = db0 + __builtin_ctz(dm);
        dm &= dm - 1;
        const int c0b = fs_blk_begin(fs, i), ln = fs_blk_len(fs, i);
        const int aa = max(o, p0), bb = min(o + ln, p1);
        oo = o;
        o += ln;
        if (aa < bb) {
          cb = c0b;
          a = aa;
          b = bb;
          have = true;
          break;
        }
      }
      uint64_t bal = __ballot(have);
      if (bal == 0) break;
      while (bal) {
        const int l = __builtin_ctzll(bal);
        bal &= bal - 1;
        const int cbl = __shfl(cb, l), ool = __shfl(oo, l);
        const int al = __shfl(a, l), bl = __shfl(b, l);
        for (int t = al + lane; t < bl; t += 64) {
          const int col = cbl + (t - ool);
          s_list[t - p0] = col;
          if (P == 0) sel_out[t] = col;
        }
      }
    }
  };
  const int per = (S + CPP - 1) / CPP;
  const int c0 = min(S, c * per), c1 = min(S, c0 + per);
  const int sub = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int NP1 = NP + 1;
  int p0 = c0, p1 = min(c1, c0 + kSplitList);
  if (DRAW) {
    expand(p0, p1);
    __syncthreads();
  }
  // drawn columns of the coordinates tb + grp + G * i, then their panel offsets [a, b)
  // (an empty run past p1); the list is read two passes ahead, the offsets one
  auto load_cols = [&](int tb, int (&jr)[CPG]) {
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      const int t = tb + grp + G * i;
      jr[i] = DRAW ? s_list[t < p1 ? t - p0 : 0] : sel_cols[t < p1 ? t : 0];
    }
  };
  auto load_offs = [&](int tb, const int (&jr)[CPG], int (&a)[CPG], int (&b)[CPG]) {
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      const int t = tb + grp + G * i;
      const size_t o = (size_t)(t < p1 ? jr[i] : 0) * NP1 + P;
      a[i] = pofs[o];
      b[i] = pofs[o + (t < p1 ? 1 : 0)];
    }
  };
  int jn[CPG], ks[CPG], ke[CPG];
  if (p0 < p1) {  // in flight while r's panel is staged
    load_cols(p0, jn);
    load_offs(p0, jn, ks, ke);
    load_cols(p0 + G * CPG, jn);
  }
  stage_r();
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads of r's panel have landed
  if ((int)threadIdx.x == nfull % 1024 && nfull * VN < len) {  // the last partial group
    T tail[VN];
#pragma unroll
    for (int e = 0; e < VN; ++e) tail[e] = nfull * VN + e < len ? r[lo + nfull * VN + e] : (T)0;
#pragma unroll
    for (int e = 0; e < VN; ++e)
      if (nfull * VN + e < len) s_r[nfull * VN + e] = tail[e];
  }
  __syncthreads();
  for (;;) {
  for (int tb = p0; tb < p1; tb += G * CPG) {
    int rw[CPG][H];
    T vw[CPG][H];
#pragma unroll
    for (int i = 0; i < CPG; ++i)
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int k = ks[i] + sub + 16 * h;
        const int kk = k < ke[i] ? k : 0;
        rw[i][h] = rowidx[kk];
        vw[i][h] = v[kk];
      }
    int ks2[CPG], ke2[CPG];
    load_offs(tb + G * CPG, jn, ks2, ke2);
    load_cols(tb + 2 * G * CPG, jn);
    // r at the window rows.  Lanes past the run read entry 0's row clamped into the panel
    // (read, not used): the index never depends on the run test, so the compiler keeps
    // every row load unconditional (a load it sinks under the test is followed by a wait
    // for every load in flight, the next pass's prefetches included).
    const unsigned rmax = (unsigned)max(len - 1, 0);
    T rv[CPG][H];
#pragma unroll
    for (int i = 0; i < CPG; ++i)
#pragma unroll
      for (int h = 0; h < H; ++h) rv[i][h] = s_r[min((unsigned)(rw[i][h] - lo), rmax)];
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      T acc = (T)0;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const T a2 = acc + vw[i][h] * rv[i][h];
        acc = ks[i] + sub + 16 * h < ke[i] ? a2 : acc;
      }
      for (int k0 = ks[i] + sub + 16 * H; k0 < ke[i]; k0 += 64) {
        int rq[4];
        T vq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 16 * u;
          const int kk = k < ke[i] ? k : 0;
          rq[u] = rowidx[kk];
          vq[u] = v[kk];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (k0 + 16 * u < ke[i]) acc += vq[u] * s_r[rq[u] - lo];
      }
      acc = sum16(acc);
      const int t = tb + grp + G * i;
      if (sub == 0 && t < p1) part[(size_t)P * ldpart + t] = acc;
    }
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      ks[i] = ks2[i];
      ke[i] = ke2[i];
    }
  }
  // the next piece of the chunk (only when it holds more than kSplitList columns)
  if (p1 >= c1) break;
  __syncthreads();  // every group is done with s_list
  p0 = p1;
  p1 = min(c1, p0 + kSplitList);
  if (DRAW) {
    expand(p0, p1);
    __syncthreads();
  }
  load_cols(p0, jn);
  load_offs(p0, jn, ks, ke);
  load_cols(p0 + G * CPG, jn);
  }
}

// S.2 (second half) + S.4 after k_dot_split: the NP partials of each drawn coordinate are
// added by sum16 (lane sub holds panel sub's), then the best response and the step; the
// moved columns' nonzeros are counted per row bin (64 entries of every moved column per
// step).  Loads are unconditional as in k_dot_split.  Same work mapping and outputs as
// k_grad_br_csc.  gnext: the draw ran in k_dot_split and the round state is not advanced
// yet, so the round's step is st->gamma_next.
template <typename T, int CPG>
__global__ void __launch_bounds__(kCscThreads)
k_br_split(const long long* __restrict__ colptr, const int* __restrict__ rowidx,
           const T* __restrict__ part, long long ldpart, int NP, T* __restrict__ x,
           const double* __restrict__ cn2, const int* __restrict__ sel_cols,
           const RoundState* __restrict__ st, T* __restrict__ dx_sel, BRParams bp, int bin_log,
           int nb, int* __restrict__ cnt, int* __restrict__ moved_wg, int gnext) {
  extern __shared__ int hist[];
  __shared__ int s_moved[kCscThreads / 64];
  for (int i = threadIdx.x; i < nb; i += kCscThreads) hist[i] = 0;
  __syncthreads();
  constexpr int G = kCscThreads / 16;
  const int sub = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const T gamma = (T)(gnext ? st->gamma_next : st->gamma_cur);
  int c0, c1;
  wg_chunk(st->S_cnt, &c0, &c1);
  int moved = 0;
  for (int tb = c0; tb < c1; tb += G * CPG) {
    int jj[CPG], kb[CPG], ke[CPG];
    T pv[CPG], xj[CPG];
    double qj[CPG];
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      const int t = tb + grp + G * i;
      const bool ok = t < c1;
      jj[i] = sel_cols[ok ? t : 0];
      pv[i] = part[ok && sub < NP ? (size_t)sub * ldpart + t : 0];
    }
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      const int t = tb + grp + G * i;
      const int j = t < c1 ? jj[i] : 0;
      xj[i] = x[j];
      qj[i] = cn2[j];
      kb[i] = (int)colptr[j];
      ke[i] = (int)colptr[j + 1];
    }
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      const int t = tb + grp + G * i;
      const T dot = sum16(t < c1 && sub < NP ? pv[i] : (T)0);
      if (t >= c1) {
        ke[i] = kb[i];  // no coordinate: no bin counts
        continue;
      }
      const T d = csc_step_v<T>(dot, xj[i], qj[i], jj[i], t, sub, gamma, x, dx_sel, bp);
      if (d != (T)0)
        moved += sub == 0;
      else
        ke[i] = kb[i];  // not moved: no bin counts
    }
    for (int o = 0;; o += 64) {
      int rr[CPG][4];
#pragma unroll
      for (int i = 0; i < CPG; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = kb[i] + o + sub + 16 * u;
          rr[i][u] = rowidx[k < ke[i] ? k : 0];
        }
      bool left = false;
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (kb[i] + o + sub + 16 * u < ke[i]) atomicAdd(&hist[rr[i][u] >> bin_log], 1);
        left |= kb[i] + o + 64 < ke[i];
      }
      if (!left) break;
    }
  }
  __syncthreads();
  flush_counts(hist, nb, moved, s_moved, cnt, moved_wg);
}

// Bin counts of the nonzeros of the columns j < n with coef[j] != 0 (same work mapping as
// the gradient kernels; used for a fresh residual).
template <typename T>
__global__ void __launch_bounds__(kCscThreads)
k_bin_hist(const long long* __restrict__ colptr, const int* __restrict__ rowidx,
           const T* __restrict__ coef, int n, int bin_log, int nb, int* __restrict__ cnt) {
  extern __shared__ int hist[];
  __shared__ int s_moved[kCscThreads / 64];
  for (int i = threadIdx.x; i < nb; i += kCscThreads) hist[i] = 0;
  __syncthreads();
  const int sub = threadIdx.x & 15;
  int c0, c1;
  wg_chunk(n, &c0, &c1);
  for (int j = c0 + (int)(threadIdx.x >> 4); j < c1; j += kCscThreads / 16) {
    if (coef[j] == (T)0) continue;
    for (long long k = colptr[j] + sub; k < colptr[j + 1]; k += 16)
      atomicAdd(&hist[rowidx[k] >> bin_log], 1);
  }
  __syncthreads();
  flush_counts(hist, nb, 0, s_moved, cnt, nullptr);
}

// cnt[w][bin] -> exclusive prefix over w inside each bin; tot[bin] = bin total.  One
// workgroup per bin; thread i takes a run of consecutive w (all its loads in flight at
// once), then a block scan orders the runs.  Block 0 also adds the moved columns of the
// round to the running statistics and, with advance (the draw ran inside the gradient
// kernel), advances the round as k_select does: drawn count, round counter, step.
template <int PER>
__global__ void __launch_bounds__(256)
k_bin_scan(int* __restrict__ cnt, int grid, int nb, int* __restrict__ tot,
           const int* __restrict__ moved_wg, RoundState* __restrict__ st, int advance) {
  __shared__ int sh[5];
  __shared__ long long s_mv[4];
  const int bin = blockIdx.x;
  const int w0 = threadIdx.x * PER;
  int c[PER];
  int sum = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    c[u] = w0 + u < grid ? cnt[(size_t)(w0 + u) * nb + bin] : 0;
    sum += c[u];
  }
  int total;
  int run = block_exclusive_scan<4>(sum, sh, &total);
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (w0 + u < grid) cnt[(size_t)(w0 + u) * nb + bin] = run;
    run += c[u];
  }
  if (threadIdx.x == 0) tot[bin] = total;
  if (blockIdx.x == 0 && moved_wg) {
    long long mv = 0;
    for (int w = threadIdx.x; w < grid; w += 256) mv += moved_wg[w];
    mv = wave_sum_i64(mv);
    if ((threadIdx.x & 63) == 0) s_mv[threadIdx.x >> 6] = mv;
    __syncthreads();
    if (threadIdx.x == 0) {
      st->moved_updates += s_mv[0] + s_mv[1] + s_mv[2] + s_mv[3];
      if (advance) {
        const double g = st->gamma_next;
        st->coord_updates += st->S_cnt;
        st->k += 1;
        st->work_ctr = 0;
        st->gamma_cur = g;
        st->gamma_next = g * (1.0 - st->gamma_mu * g);
      }
    }
  }
}

// Start of every bin's slots (exclusive scan of tot) into base[0..nb); 256 threads.
__device__ __forceinline__ void bin_starts(const int* __restrict__ tot, int nb, int* base,
                                           int* sh) {
  const int per = (nb + kCscThreads - 1) / kCscThreads;
  const int i0 = min(nb, (int)threadIdx.x * per), i1 = min(nb, i0 + per);
  int loc = 0;
  for (int i = i0; i < i1; ++i) loc += tot[i];
  int total;
  int run = block_exclusive_scan<kCscThreads / 64>(loc, sh, &total);
  for (int i = i0; i < i1; ++i) {
    base[i] = run;
    run += tot[i];
  }
}

// One fold entry: row inside its bin and the product a_ij * dx_j, stored with one 8-byte
// (FP32) or 16-byte (FP64) write.
template <typename T> struct Ent;
template <> struct alignas(8) Ent<float> {
  uint32_t row;
  float val;
};
template <> struct alignas(16) Ent<double> {
  uint64_t row;
  double val;
};
__device__ __forceinline__ void put_ent(Ent<float>* e, long long pos, uint32_t row, float val) {
  reinterpret_cast<uint2*>(e)[pos] = make_uint2(row, __float_as_uint(val));
}
__device__ __forceinline__ void put_ent(Ent<double>* e, long long pos, uint32_t row, double val) {
  reinterpret_cast<ulonglong2*>(e)[pos] =
      make_ulonglong2((unsigned long long)row, (unsigned long long)__double_as_longlong(val));
}

// Writes the entries (row within bin, a_ij * coef) of the listed columns with coef != 0
// into their bins' slots.  list == nullptr: the columns 0..count-1 with coef indexed by j;
// otherwise list[t] with coef indexed by t.  Same work mapping as the counting kernel; each
// group of 16 lanes takes 16/U columns at once and loads 16*U nonzeros of each per step,
// all before their slots are taken.
template <typename T, int U>
__global__ void __launch_bounds__(kCscThreads)
k_bin_scatter(const long long* __restrict__ colptr, const int* __restrict__ rowidx,
              const T* __restrict__ v, const int* __restrict__ list,
              const int* __restrict__ count_ptr, int count, const T* __restrict__ coef,
              int bin_log, int nb, const int* __restrict__ off, const int* __restrict__ tot,
              Ent<T>* __restrict__ ent) {
  extern __shared__ int cursor[];
  __shared__ int sh[kCscThreads / 64 + 1];
  bin_starts(tot, nb, cursor, sh);
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += kCscThreads) cursor[i] += off[(size_t)blockIdx.x * nb + i];
  __syncthreads();
  constexpr int G = kCscThreads / 16;
  constexpr int CPG = 16 / U;  // columns per group in flight
  const int sub = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const uint32_t rmask = (1u << bin_log) - 1u;
  int c0, c1;
  wg_chunk(count_ptr ? *count_ptr : count, &c0, &c1);
  // the columns t = tb + grp + G * i (the same ones, per workgroup, as the counting
  // kernels); loads are unconditional (clamped to valid positions, their values unused)
  for (int tb = c0; tb < c1; tb += G * CPG) {
    int jr[CPG], kb[CPG], ke[CPG];
    T d[CPG];
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      const int t = tb + grp + G * i;
      const int ts = t < c1 ? t : c0;
      jr[i] = list ? list[ts] : ts;
      d[i] = coef[ts];
    }
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
      kb[i] = (int)colptr[jr[i]];
      ke[i] = (int)colptr[jr[i] + 1];
    }
#pragma unroll
    for (int i = 0; i < CPG; ++i)
      if (tb + grp + G * i >= c1 || d[i] == (T)0) ke[i] = kb[i];
    for (int o = 0;; o += 16 * U) {
      int ri[CPG][U];
      T vv[CPG][U];
#pragma unroll
      for (int i = 0; i < CPG; ++i)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = kb[i] + o + sub + 16 * u;
          const int kk = k < ke[i] ? k : 0;
          ri[i][u] = rowidx[kk];
          vv[i][u] = v[kk];
        }
      bool left = false;
#pragma unroll
      for (int i = 0; i < CPG; ++i) {
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (kb[i] + o + sub + 16 * u < ke[i]) {
            const int pos = atomicAdd(&cursor[ri[i][u] >> bin_log], 1);
            put_ent(ent, pos, (uint32_t)ri[i][u] & rmask, vv[i][u] * d[i]);
          }
        left |= kb[i] + o + 16 * U < ke[i];
      }
      if (!left) break;
    }
  }
}

// Exact fixed-point accumulation in limbs: a row's cell is four signed 64-bit limbs with
// weights 2^(32k) (k = 0..3) in units of 2^-72, stored limb-major (limb k of row r at
// k * R + r, so the lanes of a wave spread over the LDS banks).  An entry's magnitude, an integer mantissa
// M times a power of two, is placed at bit s = exponent + 72 (bits below the unit are
// truncated toward zero) and split into 32-bit chunks, each added to its limb with a
// non-returning LDS atomic; a limb takes 2^31 such additions before it can overflow.
// Integer sums do not depend on the order of the additions; carries are resolved once
// when the cell is read.  Magnitudes below 2^55 are represented, per entry and per row sum:
// an entry outside that range (or Inf / NaN) is not added but reported to the caller, and a
// row sum beyond it reads as NaN, so an out-of-range fold shows up as a non-finite residual.
constexpr int kLimbs = 4;
constexpr double kLimbRange = 36028797018963968.0;  // 2^55
__device__ __forceinline__ void limb_add(long long* cell, int R, unsigned long long M, int s,
                                         bool neg) {
  if (s < 0) {
    if (s <= -64) return;
    M >>= -s;
    s = 0;
  }
  if (M == 0ull) return;
  int k = s >> 5;
  const int o = s & 31;
  // M < 2^53 and o < 32: M << o spans at most three 32-bit chunks; below 2^55 the top
  // set bit is at most bit 126, so no chunk lies beyond the top limb
  const unsigned long long lo = M << o;
  const unsigned long long hi = o ? (M >> (64 - o)) : 0ull;
  const unsigned long long ch[3] = {lo & 0xffffffffull, lo >> 32, hi};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int kk = k + i;
    if (ch[i] == 0ull || kk >= kLimbs) continue;
    const unsigned long long c = ch[i];
    atomicAdd((unsigned long long*)&cell[kk * R], neg ? 0ull - c : c);
  }
}
// Adds v to the cell; returns false (adding nothing) when |v| >= 2^55 or v is not finite.
__device__ __forceinline__ bool limb_add_val(long long* cell, int R, float v) {
  if (!(fabsf(v) < (float)kLimbRange)) return false;
  const uint32_t u = __float_as_uint(v);
  const int ex = (int)((u >> 23) & 0xffu);
  if (ex == 0) return true;  // zero or subnormal: below the unit
  const unsigned long long M = (unsigned long long)((u & 0x7fffffu) | 0x800000u);
  limb_add(cell, R, M, ex - 127 - 23 + 72, (u >> 31) != 0u);
  return true;
}
__device__ __forceinline__ bool limb_add_val(long long* cell, int R, double v) {
  if (!(fabs(v) < kLimbRange)) return false;
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int ex = (int)((u >> 52) & 0x7ffull);
  if (ex == 0) return true;
  const unsigned long long M = (u & 0xfffffffffffffull) | (1ull << 52);
  limb_add(cell, R, M, ex - 1023 - 52 + 72, (u >> 63) != 0ull);
  return true;
}
// Value of a cell in one rounding from its 128-bit two's-complement integer.
__device__ __forceinline__ double limb_value(const long long* cell, int R) {
  long long t = cell[0];
  const unsigned long long c0 = (unsigned long long)t & 0xffffffffull;
  t = cell[R] + (t >> 32);
  const unsigned long long c1 = (unsigned long long)t & 0xffffffffull;
  t = cell[2 * R] + (t >> 32);
  const unsigned long long c2 = (unsigned long long)t & 0xffffffffull;
  t = cell[3 * R] + (t >> 32);
  // the 128-bit sum is t * 2^96 + (c2, c1, c0): beyond 2^55 (t outside 32 bits) it wrapped
  if (t < -2147483648ll || t > 2147483647ll) return __longlong_as_double(0x7ff8000000000000ll);
  const long long hi = (long long)(((unsigned long long)t << 32) | c2);
  const unsigned long long lo = (c1 << 32) | c0;
  return ldexp((double)hi, 64 - 72) + ldexp((double)lo, -72);
}

// One workgroup per bin: the bin's entries are summed into limb cells in LDS (eight entry
// loads per thread in flight), then out[i] = base_scale * base[i] + cell_i for the bin's
// rows (one rounding; out may alias base; out and out64 may each be NULL).  A row that
// received an entry the cells cannot hold (see limb_add_val) is written as NaN.
// Dynamic LDS: kLimbs * R long longs of cells, then R ints of flags.
constexpr int kAccThreads = 1024;
constexpr int kAccUnroll = 8;
template <typename T, typename TB, typename TO>
__global__ void __launch_bounds__(kAccThreads)
k_bin_acc(const Ent<T>* __restrict__ ent, const int* __restrict__ tot, int bin_log, int m,
          const TB* base, double base_scale, TO* out, double* __restrict__ out64) {
  extern __shared__ long long cells[];
  __shared__ long long s_part[kAccThreads / 64];
  const int R = 1 << bin_log;
  const int bin = blockIdx.x;
  int* bad = (int*)(cells + kLimbs * R);
  for (int i = threadIdx.x; i < kLimbs * R; i += kAccThreads) cells[i] = 0;
  for (int i = threadIdx.x; i < R; i += kAccThreads) bad[i] = 0;
  long long pre = 0;
  for (int i = threadIdx.x; i < bin; i += kAccThreads) pre += tot[i];
  pre = wave_sum_i64(pre);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = pre;
  __syncthreads();
  long long start = 0;
  for (int w = 0; w < kAccThreads / 64; ++w) start += s_part[w];
  const long long end = start + tot[bin];
  for (long long e0 = start + threadIdx.x; e0 < end; e0 += kAccThreads * kAccUnroll) {
    Ent<T> en[kAccUnroll];
#pragma unroll
    for (int u = 0; u < kAccUnroll; ++u) {  // unconditional loads (past the bin: entry e0)
      const long long e = e0 + (long long)u * kAccThreads;
      en[u] = ent[e < end ? e : e0];
    }
#pragma unroll
    for (int u = 0; u < kAccUnroll; ++u) {
      const bool ok = e0 + (long long)u * kAccThreads < end;
      const int row = ok ? (int)en[u].row : 0;
      if (!limb_add_val(&cells[row], R, ok ? en[u].val : (T)0)) atomicOr(&bad[row], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += kAccThreads) {
    const int row = bin * R + i;
    if (row >= m) break;
    const double s = bad[i] ? __longlong_as_double(0x7ff8000000000000ll)
                            : base_scale * (double)base[row] + limb_value(&cells[i], R);
    if (out) out[row] = (TO)s;
    if (out64) out64[row] = s;
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_probe_csc(const long long* __restrict__ colptr, const int* __restrict__ rowidx,
            const T* __restrict__ v, const double* __restrict__ r64, const T* __restrict__ x,
            int n, const double* __restrict__ cn2, BRParams bp, double* __restrict__ wmax,
            double* __restrict__ wsum, int* __restrict__ wcnt) {
  const int sub = threadIdx.x & 15;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
  double mx = 0.0, sm = 0.0;
  int cnt = 0;
  const int ngroup = gridDim.x * 16;
  for (int j = blockIdx.x * 16 + (threadIdx.x >> 4); j < n; j += ngroup) {
    const double dot = csc_col_dot<T, double, double>(colptr, rowidx, v, r64, j, sub);
    if (sub == 0) {
      const double xj = (double)x[j];
      double g = dot - bp.c2 * xj;
      if (bp.reg) g -= bp.lam * dh_minus<double>(xj, bp);
      const double q = cn2[j] + bp.tau;
      const double xh = soft_clip<double>(xj - g / q, bp.lam_eta / q, bp.beta);
      const double y = soft_clip<double>(xj - g, bp.lam_eta, bp.beta);
      mx = fmax(mx, fabs(xh - xj));
      sm += (xj - y) * (xj - y);
      cnt += (xh != 0.0);
    }
  }
  // lanes 0, 16, 32, 48 hold values; fixed-order combination inside the wave
  mx = wave_max(mx);
  sm = wave_sum(sm);
  const int c = (int)wave_sum_i64((long long)cnt);
  if (lane == 0) {
    wmax[gw] = mx;
    wsum[gw] = sm;
    wcnt[gw] = c;
  }
}

// Bin scan, scatter and accumulation of a fold whose counts are in p->d_bin_cnt.
template <typename T, typename TB, typename TO>
void bin_fold(sca_problem* p, const int* list, const int* count_ptr, int count, const T* coef,
              const int* moved_wg, const TB* base, double base_scale, TO* out, double* out64,
              hipStream_t s, int advance = 0) {
  const int nb = p->bin_nb, grid = p->bin_grid;
  if (grid <= 256 * 4)
    hipLaunchKernelGGL(k_bin_scan<4>, dim3(nb), dim3(256), 0, s, p->d_bin_cnt, grid, nb,
                       p->d_bin_tot, moved_wg, p->d_state, advance);
  else
    hipLaunchKernelGGL(k_bin_scan<kBinGridMax / 256>, dim3(nb), dim3(256), 0, s, p->d_bin_cnt,
                       grid, nb, p->d_bin_tot, moved_wg, p->d_state, advance);
  if (p->bin_unroll == 2)
    hipLaunchKernelGGL((k_bin_scatter<T, 2>), dim3(grid), dim3(kCscThreads), sizeof(int) * nb, s,
                       (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                       (const T*)p->csc_vals, list, count_ptr, count, coef, p->bin_log, nb,
                       (const int*)p->d_bin_cnt, (const int*)p->d_bin_tot, (Ent<T>*)p->d_ent);
  else if (p->bin_unroll == 4)
    hipLaunchKernelGGL((k_bin_scatter<T, 4>), dim3(grid), dim3(kCscThreads), sizeof(int) * nb, s,
                       (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                       (const T*)p->csc_vals, list, count_ptr, count, coef, p->bin_log, nb,
                       (const int*)p->d_bin_cnt, (const int*)p->d_bin_tot, (Ent<T>*)p->d_ent);
  else
    hipLaunchKernelGGL((k_bin_scatter<T, 8>), dim3(grid), dim3(kCscThreads), sizeof(int) * nb, s,
                       (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                       (const T*)p->csc_vals, list, count_ptr, count, coef, p->bin_log, nb,
                       (const int*)p->d_bin_cnt, (const int*)p->d_bin_tot, (Ent<T>*)p->d_ent);
  hipLaunchKernelGGL((k_bin_acc<T, TB, TO>), dim3(nb), dim3(kAccThreads),
                     (sizeof(long long) * kLimbs + sizeof(int)) * ((size_t)1 << p->bin_log), s,
                     (const Ent<T>*)p->d_ent, (const int*)p->d_bin_tot, p->bin_log, (int)p->m,
                     base, base_scale, out, out64);
}

template <typename T, int U>
void grad_launch(sca_problem* p, T* x, const T* r, const BRParams& bp, hipStream_t s) {
  hipLaunchKernelGGL((k_grad_br_csc<T, U>), dim3(p->bin_grid), dim3(kCscThreads),
                     sizeof(int) * p->bin_nb, s, (const long long*)p->csc_colptr,
                     (const int*)p->csc_rowidx, (const T*)p->csc_vals, r, x, p->d_cn2,
                     p->d_sel_cols, (const RoundState*)p->d_state, (T*)p->d_dx_sel, bp,
                     p->bin_log, p->bin_nb, p->d_bin_cnt, p->d_bin_moved);
}

// fs.on (panel split only): the block draw runs inside k_dot_split.
template <typename T>
void grad_any(sca_problem* p, T* x, const T* r, const BRParams& bp, const FusedSel& fs,
              hipStream_t s) {
  if (p->sp_np > 0) {
    constexpr int CPG = sizeof(T) == 4 ? 8 : 4;
    const int NP = p->sp_np, CPP = std::max(1, p->ncu / NP);
    const long long ldpart = std::max<long long>(1, p->n);
    if (fs.on)
      hipLaunchKernelGGL((k_dot_split<T, CPG, true>), dim3(NP * CPP), dim3(1024), 0, s,
                         (const int*)p->d_pofs, (const int*)p->csc_rowidx, (const T*)p->csc_vals,
                         r, p->d_sel_cols, p->d_state, (int)p->m, NP, p->sp_pe, CPP,
                         (T*)p->d_sp_part, ldpart, fs, p->d_sel_cols);
    else
      hipLaunchKernelGGL((k_dot_split<T, CPG, false>), dim3(NP * CPP), dim3(1024), 0, s,
                         (const int*)p->d_pofs, (const int*)p->csc_rowidx, (const T*)p->csc_vals,
                         r, p->d_sel_cols, p->d_state, (int)p->m, NP, p->sp_pe, CPP,
                         (T*)p->d_sp_part, ldpart, fs, p->d_sel_cols);
    hipLaunchKernelGGL((k_br_split<T, CPG>), dim3(p->bin_grid), dim3(kCscThreads),
                       sizeof(int) * p->bin_nb, s, (const long long*)p->csc_colptr,
                       (const int*)p->csc_rowidx, (const T*)p->d_sp_part, ldpart, NP, x,
                       p->d_cn2, p->d_sel_cols, (const RoundState*)p->d_state, (T*)p->d_dx_sel,
                       bp, p->bin_log, p->bin_nb, p->d_bin_cnt, p->d_bin_moved, fs.on);
  } else if (p->bin_panel) {
    hipLaunchKernelGGL((k_grad_br_cscp<T, sizeof(T) == 4 ? 8 : 4>), dim3(p->bin_grid),
                       dim3(kPanelThreads), 0, s,
                       (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                       (const T*)p->csc_vals, r, x, p->d_cn2, p->d_sel_cols,
                       (const RoundState*)p->d_state, (T*)p->d_dx_sel, bp, (int)p->m,
                       p->bin_log, p->bin_nb, p->d_bin_cnt, p->d_bin_moved);
  } else if (p->bin_unroll == 2) {
    grad_launch<T, 2>(p, x, r, bp, s);
  } else if (p->bin_unroll == 4) {
    grad_launch<T, 4>(p, x, r, bp, s);
  } else {
    grad_launch<T, 8>(p, x, r, bp, s);
  }
}

// The panel-split gradient draws the round's blocks itself when every thread of its
// 1024-thread workgroups owns at most 32 of them.
template <typename T>
void round_csc(sca_problem* p, const sca_opts* o, T* x, T* r, hipStream_t s, uint64_t Tthr,
               const BRParams& bp) {
  FusedSel fs{p->d_bp, (int)p->nblocks, 0, o->seed, Tthr, o->instance, p->blk_uniform,
              (int)p->n};
  fs.on = p->sp_np > 0 && p->nblocks <= kFusedSelBlocks;
  if (!fs.on) {
    prof_begin(p, s, SCA_K_SELECT);
    launch_select(p, o, Tthr, s);
    prof_end(p, s, 0.0);
  }
  prof_begin(p, s, SCA_K_GRAD);
  grad_any<T>(p, x, r, bp, fs, s);
  prof_end(p, s, 0.0);
  prof_begin(p, s, SCA_K_FOLD);
  int* S_ptr = (int*)((char*)p->d_state + offsetof(RoundState, S_cnt));
  bin_fold<T, T, T>(p, p->d_sel_cols, S_ptr, 0, (const T*)p->d_dx_sel, p->d_bin_moved, r, 1.0,
                    r, (double*)nullptr, s, fs.on);
  prof_end(p, s, 0.0);
}

template <typename T>
void residual_csc(sca_problem* p, const T* x, T* r_out, hipStream_t s) {
  hipLaunchKernelGGL(k_bin_hist<T>, dim3(p->bin_grid), dim3(kCscThreads),
                     sizeof(int) * p->bin_nb, s, (const long long*)p->csc_colptr,
                     (const int*)p->csc_rowidx, x, (int)p->n, p->bin_log, p->bin_nb,
                     p->d_bin_cnt);
  bin_fold<T, T, T>(p, (const int*)nullptr, (const int*)nullptr, (int)p->n, x,
                    (const int*)nullptr, (const T*)p->b, -1.0, r_out, p->d_r64, s);
}

}  // namespace

// ------------------------------------------------------------------ hooks used by the API
void sca::launch_colnorm2_csc(sca_problem* p, hipStream_t s) {
  const int grid = std::max(1, std::min<int>((int)((p->n + 255) / 256), 8 * p->ncu));
  if (p->dtype == SCA_F32)
    hipLaunchKernelGGL(k_colnorm2_csc<float>, dim3(grid), dim3(256), 0, s,
                       (const long long*)p->csc_colptr, (const float*)p->csc_vals, (int)p->n,
                       p->d_cn2);
  else
    hipLaunchKernelGGL(k_colnorm2_csc<double>, dim3(grid), dim3(256), 0, s,
                       (const long long*)p->csc_colptr, (const double*)p->csc_vals, (int)p->n,
                       p->d_cn2);
}

void sca::launch_round_csc(sca_problem* p, const sca_opts* o, void* x, void* r, hipStream_t s,
                           uint64_t Tthr, const BRParams& bp) {
  if (p->dtype == SCA_F32)
    round_csc<float>(p, o, (float*)x, (float*)r, s, Tthr, bp);
  else
    round_csc<double>(p, o, (double*)x, (double*)r, s, Tthr, bp);
}

void sca::launch_residual_csc(sca_problem* p, const void* x, void* r_out, hipStream_t s) {
  if (p->dtype == SCA_F32)
    residual_csc<float>(p, (const float*)x, (float*)r_out, s);
  else
    residual_csc<double>(p, (const double*)x, (double*)r_out, s);
}

void sca::launch_probe_csc(sca_problem* p, const void* x, const BRParams& bp, hipStream_t s) {
  const int grid = p->probe_waves / 4;
  if (p->dtype == SCA_F32)
    hipLaunchKernelGGL(k_probe_csc<float>, dim3(grid), dim3(256), 0, s,
                       (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                       (const float*)p->csc_vals, (const double*)p->d_r64, (const float*)x,
                       (int)p->n, (const double*)p->d_cn2, bp, p->d_wmax, p->d_wsum, p->d_wcnt);
  else
    hipLaunchKernelGGL(k_probe_csc<double>, dim3(grid), dim3(256), 0, s,
                       (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                       (const double*)p->csc_vals, (const double*)p->d_r64, (const double*)x,
                       (int)p->n, (const double*)p->d_cn2, bp, p->d_wmax, p->d_wsum, p->d_wcnt);
}

// ------------------------------------------------------------------ create
template <typename T>
static sca_status build_csc(sca_problem* p, const long long* rowptr, const int32_t* colidx,
                            const T* vals, hipStream_t s) {
  const int m = (int)p->m, n = (int)p->n;
  const long long nnz = p->nnz;
  sca_status st;
  int *colcnt = nullptr, *flags = nullptr, *tmp_row = nullptr;
  long long* tmp_src = nullptr;
  auto cleanup = [&]() {
    if (colcnt) (void)hipFree(colcnt);
    if (flags) (void)hipFree(flags);
    if (tmp_row) (void)hipFree(tmp_row);
    if (tmp_src) (void)hipFree(tmp_src);
  };
  if ((st = dev_alloc((void**)&colcnt, sizeof(int) * (size_t)(n + 1))) != SCA_OK ||
      (st = dev_alloc((void**)&flags, sizeof(int) * 4)) != SCA_OK ||
      (st = dev_alloc((void**)&tmp_row, sizeof(int) * (size_t)std::max(1ll, nnz))) != SCA_OK ||
      (st = dev_alloc((void**)&tmp_src, sizeof(long long) * (size_t)std::max(1ll, nnz))) != SCA_OK ||
      (st = dev_alloc((void**)&p->csc_colptr, sizeof(long long) * (size_t)(n + 1))) != SCA_OK ||
      (st = dev_alloc((void**)&p->csc_rowidx, sizeof(int) * (size_t)std::max(1ll, nnz))) != SCA_OK ||
      (st = dev_alloc((void**)&p->csc_vals, sizeof(T) * (size_t)std::max(1ll, nnz))) != SCA_OK ||
      (st = dev_alloc((void**)&p->d_bin_cnt,
                      sizeof(int) * (size_t)p->bin_grid * p->bin_nb)) != SCA_OK ||
      (st = dev_alloc((void**)&p->d_bin_tot, sizeof(int) * (size_t)p->bin_nb)) != SCA_OK ||
      (st = dev_alloc((void**)&p->d_bin_moved, sizeof(int) * (size_t)p->bin_grid)) != SCA_OK ||
      (st = dev_alloc((void**)&p->d_ent, sizeof(Ent<T>) * (size_t)std::max(1ll, nnz))) != SCA_OK) {
    cleanup();
    return st;
  }
  // the row pointer is validated on the host
  std::vector<long long> hrp(m + 1);
  if (hipMemcpyAsync(hrp.data(), rowptr, sizeof(long long) * (m + 1), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return set_error(SCA_EHIP, "copy of rowptr failed");
  }
  if (hrp[0] != 0 || hrp[m] != nnz) {
    cleanup();
    return set_error(SCA_EINVAL, "rowptr must start at 0 and end at nnz");
  }
  for (int i = 0; i < m; ++i)
    if (hrp[i + 1] < hrp[i]) {
      cleanup();
      return set_error(SCA_EINVAL, "rowptr is not ascending");
    }
  (void)hipMemsetAsync(colcnt, 0, sizeof(int) * (size_t)(n + 1), s);
  (void)hipMemsetAsync(flags, 0, sizeof(int) * 4, s);
  const int g = 8 * p->ncu;
  hipLaunchKernelGGL(k_count_cols, dim3(g), dim3(256), 0, s, colidx, nnz, n, colcnt, flags);
  std::vector<int> hc(n + 1);
  int hbad = 0;
  if (hipMemcpyAsync(hc.data(), colcnt, sizeof(int) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&hbad, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return set_error(SCA_EHIP, "column count failed");
  }
  if (hbad) {
    cleanup();
    return set_error(SCA_EINVAL, "colidx holds an index outside [0, n)");
  }
  std::vector<long long> hcp(n + 1);
  hcp[0] = 0;
  for (int j = 0; j < n; ++j) hcp[j + 1] = hcp[j] + hc[j];
  if (hipMemcpyAsync(p->csc_colptr, hcp.data(), sizeof(long long) * (n + 1),
                     hipMemcpyHostToDevice, s) != hipSuccess) {
    cleanup();
    return set_error(SCA_EHIP, "copy of colptr failed");
  }
  (void)hipMemsetAsync(colcnt, 0, sizeof(int) * (size_t)(n + 1), s);
  hipLaunchKernelGGL(k_scatter_cols<T>, dim3(g), dim3(256), 0, s, rowptr, colidx, vals, m,
                     (const long long*)p->csc_colptr, colcnt, tmp_row, tmp_src);
  hipLaunchKernelGGL(k_sort_cols<T>, dim3(g), dim3(256), 0, s, (const long long*)p->csc_colptr, n,
                     (const int*)tmp_row, (const long long*)tmp_src, vals, p->csc_rowidx,
                     (T*)p->csc_vals, flags + 1);
  int hdup = 0;
  if (hipMemcpyAsync(&hdup, flags + 1, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return set_error(SCA_EHIP, "CSC conversion failed: %s", hipGetErrorString(hipGetLastError()));
  }
  cleanup();
  if (hdup) return set_error(SCA_EINVAL, "CSR holds a repeated (row, column) entry");
  return SCA_OK;
}

// Panel-split gradient set-up: panels of at most kSplitPanelBytes of r; problems that need
// more than kSplitMaxPanels, or whose offsets and partials do not fit in device memory, keep
// the panel-walk (or gather) gradient.
static sca_status split_setup(sca_problem* p, hipStream_t s) {
  const int64_t PR = kSplitPanelBytes / (int64_t)p->esize;
  const int64_t NP = (p->m + PR - 1) / PR;
  if (NP < 1 || NP > kSplitMaxPanels) return SCA_OK;
  const int64_t PE = ((p->m + NP - 1) / NP + 63) / 64 * 64;
  const size_t n1 = (size_t)std::max<int64_t>(1, p->n);
  if (dev_alloc((void**)&p->d_pofs, sizeof(int) * n1 * (size_t)(NP + 1)) != SCA_OK ||
      dev_alloc(&p->d_sp_part, p->esize * n1 * (size_t)NP) != SCA_OK) {
    if (p->d_pofs) (void)hipFree(p->d_pofs);
    if (p->d_sp_part) (void)hipFree(p->d_sp_part);
    p->d_pofs = nullptr;
    p->d_sp_part = nullptr;
    return SCA_OK;  // the panel-walk gradient needs neither
  }
  if (p->n > 0) {
    const int grid = (int)std::min<int64_t>((p->n + 255) / 256, 8 * (int64_t)p->ncu);
    hipLaunchKernelGGL(k_panel_offsets, dim3(grid), dim3(256), 0, s,
                       (const long long*)p->csc_colptr, (const int*)p->csc_rowidx, (int)p->n,
                       (int)NP, (int)PE, p->d_pofs);
    if (hipGetLastError() != hipSuccess) return set_error(SCA_EHIP, "panel offsets failed");
  }
  p->sp_np = (int)NP;
  p->sp_pe = (int)PE;
  return SCA_OK;
}

extern "C" sca_status sca_problem_create_csr(sca_problem** out, sca_dtype dtype, int64_t m,
                                             int64_t n, int64_t nnz, const int64_t* rowptr,
                                             const int32_t* colidx, const void* vals,
                                             const void* b, double lambda, double c, double beta,
                                             const int64_t* block_ptr, int64_t nblocks,
                                             void* stream) {
  if (!out) return set_error(SCA_EINVAL, "out is NULL");
  *out = nullptr;
  sca_status st = validate_problem_args(dtype, m, n, b, lambda, c, beta, block_ptr, nblocks);
  if (st != SCA_OK) return st;
  if (nnz < 0 || nnz > (int64_t)INT32_MAX)
    return set_error(SCA_EINVAL, "nnz out of range [0, 2^31)");
  if (m > ((int64_t)kMaxBins << kBinMaxLog))
    return set_error(SCA_EINVAL, "the sparse path takes m <= %lld rows",
                     (long long)((int64_t)kMaxBins << kBinMaxLog));
  if (!rowptr || (nnz > 0 && (!colidx || !vals)))
    return set_error(SCA_EINVAL, "rowptr, colidx or vals is NULL");
  sca_problem* p = new (std::nothrow) sca_problem();
  if (!p) return set_error(SCA_ENOMEM, "host allocation failed");
  p->dtype = dtype;
  p->esize = dtype == SCA_F32 ? 4 : 8;
  p->m = m;
  p->n = n;
  p->lda = 0;
  p->A = nullptr;
  p->b = b;
  p->lam = lambda;
  p->c = c;
  p->beta = beta;
  p->nblocks = nblocks;
  p->sparse = true;
  p->nnz = nnz;
  p->ncu = device_cu_count();
  // bins of R = 2^bin_log rows, at most 256 bins while 64 <= R <= 1024 (one accumulation
  // workgroup per bin: 1e5 rows give 196 bins of 512 rows)
  int lg = kBinMinLog;
  while (lg < kBinMaxLog && ((int64_t)1 << lg) * 256 < m) ++lg;
  p->bin_log = lg;
  p->bin_nb = (int)((m + ((int64_t)1 << lg) - 1) >> lg);
  p->bin_grid = std::min(kBinGridMax, p->ncu);
  p->bin_panel = p->bin_nb <= kPanelMaxBins && nnz < ((int64_t)1 << 31);
  const double per_col = n > 0 ? (double)nnz / (double)n : 0.0;
  p->bin_unroll = per_col <= 32.0 ? 2 : per_col <= 64.0 ? 4 : 8;
  hipStream_t s = (hipStream_t)stream;
  if ((st = alloc_workspace(p, block_ptr)) == SCA_OK) {
    st = dtype == SCA_F32
             ? build_csc<float>(p, (const long long*)rowptr, colidx, (const float*)vals, s)
             : build_csc<double>(p, (const long long*)rowptr, colidx, (const double*)vals, s);
  }
  if (st == SCA_OK) st = split_setup(p, s);
  if (st == SCA_OK) st = finish_create(p, s);
  if (st != SCA_OK) {
    free_workspace(p);
    delete p;
    return st;
  }
  *out = p;
  return SCA_OK;
}
