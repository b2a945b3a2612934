// gfx950 kernels of one SCA round over a dense column-major A, plus the FP64
// reductions used for checks.  All kernels are deterministic: no floating-point
// atomics, every sum has a fixed order; integer atomics only hand out work.
#pragma once
#include "sca_device.h"

namespace sca {

// Per-problem device state, updated by the kernels of a round.
struct RoundState {
  long long k;              // index of the next round to run
  long long coord_updates;  // sum of drawn coordinates over the rounds run
  long long moved_updates;  // sum of moved coordinates (columns folded) over the rounds run
  double gamma_cur;         // step of the round in flight
  double gamma_next;        // step of the following round
  double gamma_mu;          // diminishing-rule parameter (0 = fixed step)
  int S_cnt;                // coordinates drawn in the round in flight
  int work_ctr;             // next work item of the gradient kernel
  int J_cnt;                // entries of the compacted list (moved coordinates)
  int G;                    // fold: list entries per column group
  int ngroups;              // fold: number of column groups
  int n_all;                // n (length of a compaction over every coordinate)
};

// Scalars of the best response (subproblem (2) in closed form).
struct BRParams {
  double tau;      // proximal weight
  double lam;      // lambda
  double lam_eta;  // lambda * eta: soft-threshold level before division by q
  double c2;       // 2c
  double beta;     // box bound (inf = none)
  double theta;    // regulariser shape
  double eta;      // slope of h at 0
  int reg;         // 0 l1, 1 exp, 2 log
};

constexpr int kChunk = 1024;   // compaction chunk (one 1024-thread workgroup)
constexpr int kMaxGroups = 128; // fold: upper bound on column groups per call

// Derivative of h^- = eta|x| - h (the linearised concave part of the DC regularisers).
template <typename T> __device__ __forceinline__ T dh_minus(T x, const BRParams& p) {
  const T ax = fabs(x);
  T d;
  if (p.reg == 1) {
    d = (T)p.theta * ((T)1 - exp(-(T)p.theta * ax));
  } else {
    d = (T)p.eta * ((T)p.theta * ax) / ((T)1 + (T)p.theta * ax);
  }
  return x > (T)0 ? d : (x < (T)0 ? -d : (T)0);
}

template <typename T> __device__ __forceinline__ T h_value(T x, const BRParams& p) {
  const T ax = fabs(x);
  if (p.reg == 0) return ax;
  if (p.reg == 1) return (T)1 - exp(-(T)p.theta * ax);
  return log1p((T)p.theta * ax) / (T)log1p(p.theta);
}

// clip(soft(v, thr), -beta, beta)
template <typename T> __device__ __forceinline__ T soft_clip(T v, T thr, T beta) {
  const T av = fabs(v) - thr;
  T t = av > (T)0 ? copysign(av, v) : (T)0;
  return fmin(fmax(t, -beta), beta);
}

// Dot product of one column (m rows, 16-byte aligned) with r, by one wave64; every lane
// returns the sum.  U independent 16-byte loads per lane are kept in flight.
template <typename TA, typename TR, typename Acc, int U>
__device__ __forceinline__ Acc col_dot(const TA* __restrict__ col, const TR* __restrict__ r,
                                       int m, int lane) {
  typedef typename V16<TA>::v VA;
  constexpr int VN = V16<TA>::N;
  const int nvec = m / VN;
  const VA* __restrict__ cv = reinterpret_cast<const VA*>(col);
  Acc acc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) acc[u] = (Acc)0;
  int i = lane;
  for (; i + 64 * (U - 1) < nvec; i += 64 * U) {
    VA a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = __builtin_nontemporal_load(cv + i + 64 * u);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int base = (i + 64 * u) * VN;
      if constexpr (sizeof(TR) == sizeof(TA)) {
        const VA rv = *reinterpret_cast<const VA*>(r + base);
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[u] += (Acc)a[u][e] * (Acc)rv[e];
      } else {
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[u] += (Acc)a[u][e] * (Acc)r[base + e];
      }
    }
  }
  for (; i < nvec; i += 64) {
    const VA a = __builtin_nontemporal_load(cv + i);
#pragma unroll
    for (int e = 0; e < VN; ++e) acc[0] += (Acc)a[e] * (Acc)r[i * VN + e];
  }
  Acc s = acc[0];
#pragma unroll
  for (int u = 1; u < U; ++u) s += acc[u];
  const int tr = nvec * VN + lane;
  if (tr < m) s += (Acc)col[tr] * (Acc)r[tr];
  return wave_sum(s);
}

// ------------------------------------------------------------------ set-up kernels
template <typename T>
__global__ void __launch_bounds__(256) k_colnorm2(const T* __restrict__ A, long long lda, int m,
                                                  int n, double* __restrict__ cn2) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * 4;
  for (int j = blockIdx.x * 4 + (threadIdx.x >> 6); j < n; j += nw) {
    const T* col = A + (size_t)j * lda;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double v = (double)col[i];
      s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) cn2[j] = s;
  }
}

template <typename T>
static __global__ void k_count_nonfinite(const T* __restrict__ v, long long len, int* __restrict__ bad) {
  int local = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < len;
       i += (long long)gridDim.x * blockDim.x)
    local |= !isfinite((double)v[i]);
  if (local) atomicOr(bad, 1);
}

static __global__ void k_init_state(RoundState* st, long long k, double gamma, double mu, int n_all,
                             int reset_updates) {
  st->k = k;
  if (reset_updates) {
    st->coord_updates = 0;
    st->moved_updates = 0;
  }
  st->gamma_cur = gamma;
  st->gamma_next = gamma;
  st->gamma_mu = mu;
  st->S_cnt = 0;
  st->work_ctr = 0;
  st->J_cnt = 0;
  st->G = 1;
  st->ngroups = 0;
  st->n_all = n_all;
}

// ------------------------------------------------------------------ S.1: block draw
// One 1024-thread workgroup.  The block pointer is first staged in LDS (when it fits) and
// the state fields are loaded at the start, so the draw costs few memory latencies.  Each
// thread owns a contiguous range of blocks; two block scans give every drawn block its rank
// and its first output position, so the drawn coordinates are listed in ascending order.
// When the drawn blocks fit the shared list (kSelList), waves then write each drawn
// block's coordinates with coalesced stores; otherwise every thread writes its own blocks.
// Also advances the round counter and the step of the diminishing rule, and resets the
// gradient work counter.  (A grid of workgroups with a last-arriver listing measured slower
// here: its device-scope fences cost more than the draws they spread.)
constexpr int kSelList = 4096;
constexpr int kSelExpandCols = 16384;  // expected drawn columns from which the grid expands
constexpr int kSelBp = 4096;  // block pointers staged in LDS when nblocks < kSelBp

template <typename BP>
__device__ __forceinline__ void select_run(int nblocks, BP bp, uint64_t seed, uint32_t inst,
                                           uint64_t T, RoundState* __restrict__ st,
                                           int* __restrict__ sel_cols, int* sh, int* s_blk,
                                           int* s_off, int2* __restrict__ blk_out) {
  const long long k = st->k;
  double g_next = 0.0, g_mu = 0.0;
  long long upd = 0;
  if (threadIdx.x == 0) {  // loaded now so that their latency overlaps the draws
    g_next = st->gamma_next;
    g_mu = st->gamma_mu;
    upd = st->coord_updates;
  }
  const int per = (nblocks + 1023) / 1024;
  const int b0 = min(nblocks, (int)threadIdx.x * per);
  const int b1 = min(nblocks, b0 + per);
  int cnt = 0, nsel = 0;
  uint32_t mask = 0;  // drawn flags of the first 32 owned blocks
  for (int i = b0; i < b1; ++i) {
    if (block_drawn((uint32_t)i, (uint64_t)k, inst, seed, T)) {
      cnt += bp[i + 1] - bp[i];
      ++nsel;
      if (i - b0 < 32) mask |= 1u << (i - b0);
    }
  }
  int total, nsel_total;
  int off = block_exclusive_scan_1024(cnt, sh, &total);
  int rank = block_exclusive_scan_1024(nsel, sh, &nsel_total);
  const bool listed = nsel_total <= kSelList && per <= 32;
  if (listed) {
    for (int i = b0; i < b1; ++i) {
      if (mask & (1u << (i - b0))) {
        s_blk[rank] = i;
        s_off[rank] = off;
        ++rank;
        off += bp[i + 1] - bp[i];
      }
    }
    __syncthreads();
    if (blk_out) {  // k_select_expand writes the columns with the whole grid
      for (int q = threadIdx.x; q < nsel_total; q += 1024)
        blk_out[q] = make_int2(s_blk[q], s_off[q]);
      if (threadIdx.x == 0) blk_out[kSelList].x = nsel_total;
    } else {
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      for (int q = wave; q < nsel_total; q += 16) {
        const int i = s_blk[q], o = s_off[q];
        const int c0 = bp[i], len = bp[i + 1] - c0;
        for (int c = lane; c < len; c += 64) sel_cols[o + c] = c0 + c;
      }
    }
  } else {
    for (int i = b0; i < b1; ++i) {
      if (block_drawn((uint32_t)i, (uint64_t)k, inst, seed, T)) {
        for (int c = bp[i]; c < bp[i + 1]; ++c) sel_cols[off++] = c;
      }
    }
    if (blk_out && threadIdx.x == 0) blk_out[kSelList].x = 0;  // nothing left to expand
  }
  if (threadIdx.x == 0) {
    st->S_cnt = total;
    st->work_ctr = 0;
    st->coord_updates = upd + total;
    st->k = k + 1;
    st->gamma_cur = g_next;
    st->gamma_next = g_next * (1.0 - g_mu * g_next);
  }
}

// blk_out (may be NULL): when given and the drawn blocks fit the shared list, the drawn
// blocks and their first list positions go to blk_out[0..nsel) and nsel to
// blk_out[kSelList].x instead of the columns (k_select_expand writes those).
static __global__ void __launch_bounds__(1024) k_select(int nblocks, const int* __restrict__ bp,
                                                        uint64_t seed, uint32_t inst, uint64_t T,
                                                        RoundState* __restrict__ st,
                                                        int* __restrict__ sel_cols,
                                                        int2* __restrict__ blk_out) {
  __shared__ int sh[17];
  __shared__ int s_blk[kSelList];
  __shared__ int s_off[kSelList];
  __shared__ int s_bp[kSelBp];
  if (nblocks < kSelBp) {
    // all loads first (an index past nblocks reads bp[nblocks], not stored), then the stores
    int v[kSelBp / 1024];
#pragma unroll
    for (int u = 0; u < kSelBp / 1024; ++u) v[u] = bp[min((int)threadIdx.x + 1024 * u, nblocks)];
#pragma unroll
    for (int u = 0; u < kSelBp / 1024; ++u) {
      const int i = (int)threadIdx.x + 1024 * u;
      if (i <= nblocks) s_bp[i] = v[u];
    }
    __syncthreads();
    select_run(nblocks, (const int*)s_bp, seed, inst, T, st, sel_cols, sh, s_blk, s_off,
               blk_out);
  } else {
    select_run(nblocks, bp, seed, inst, T, st, sel_cols, sh, s_blk, s_off, blk_out);
  }
}

// The columns of the blocks listed by k_select in blk (count in blk[kSelList].x): wave v of
// workgroup g takes listed blocks 4g + v, 4g + v + 4G, ... and writes their columns at
// their list positions with coalesced stores.
static __global__ void __launch_bounds__(256) k_select_expand(const int2* __restrict__ blk,
                                                              const int* __restrict__ bp,
                                                              int* __restrict__ sel_cols) {
  const int n = blk[kSelList].x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = blockIdx.x * 4 + wave; q < n; q += gridDim.x * 4) {
    const int2 e = blk[q];
    const int c0 = bp[e.x], len = bp[e.x + 1] - c0;
    for (int c = lane; c < len; c += 64) sel_cols[e.y + c] = c0 + c;
  }
}

static __global__ void k_select_mask(int nblocks, uint64_t seed, uint32_t inst, uint64_t T, long long k,
                              uint8_t* __restrict__ mask) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nblocks; i += gridDim.x * blockDim.x)
    mask[i] = block_drawn((uint32_t)i, (uint64_t)k, inst, seed, T) ? 1 : 0;
}

static __global__ void k_philox(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                         long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    uint32_t c[4] = {in[6 * i], in[6 * i + 1], in[6 * i + 2], in[6 * i + 3]};
    philox4x32_10(c, in[6 * i + 4], in[6 * i + 5]);
    for (int w = 0; w < 4; ++w) out[4 * i + w] = c[w];
  }
}

// ------------------------------------------------------------------ S.2 + S.4
// One wave per drawn coordinate j (work handed out by an integer counter, next item
// prefetched): g_j = a_j^T r streamed from HBM, then the closed-form best response and
// the relaxed step.  dx_sel[t] receives the move of the t-th drawn coordinate.
template <typename T, int U>
__global__ void __launch_bounds__(256)
k_grad_br(const T* __restrict__ A, long long lda, int m, const T* __restrict__ r,
          T* __restrict__ x, const double* __restrict__ cn2, const int* __restrict__ sel_cols,
          RoundState* __restrict__ st, T* __restrict__ dx_sel, BRParams bp) {
  const int lane = threadIdx.x & 63;
  const int S = st->S_cnt;
  const T gamma = (T)st->gamma_cur;
  int t = 0;
  if (lane == 0) t = atomicAdd(&st->work_ctr, 1);
  t = __shfl(t, 0, 64);
  while (t < S) {
    int tn = 0;
    if (lane == 0) tn = atomicAdd(&st->work_ctr, 1);
    const int j = sel_cols[t];
    const T dot = col_dot<T, T, T, U>(A + (size_t)j * lda, r, m, lane);
    if (lane == 0) {
      const T xj = x[j];
      T g = dot - (T)bp.c2 * xj;
      if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
      const T q = (T)(cn2[j] + bp.tau);
      const T xh = soft_clip<T>(xj - g / q, (T)bp.lam_eta / q, (T)bp.beta);
      const T d = gamma * (xh - xj);
      x[j] = xj + d;
      dx_sel[t] = d;
    }
    t = __shfl(tn, 0, 64);
  }
}

// Workgroup variant: 256 threads walk down C drawn columns together (16-byte loads; one
// 4 KiB contiguous segment per column and step), reusing each residual load across the C
// columns; U row steps are kept in flight.  Groups of C consecutive drawn coordinates are
// handed out by an integer counter.  The per-thread partial dots are reduced in a fixed
// order (wave butterfly, then the four waves in order) before the best response.
template <typename T, int C, int U, bool NT = true>
__global__ void __launch_bounds__(256)
k_grad_br_wg(const T* __restrict__ A, long long lda, int m, const T* __restrict__ r,
             T* __restrict__ x, const double* __restrict__ cn2, const int* __restrict__ sel_cols,
             RoundState* __restrict__ st, T* __restrict__ dx_sel, BRParams bp) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  constexpr int ROWS = 256 * VN;  // rows per step of the workgroup
  __shared__ T red[4][C];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int S = st->S_cnt;
  const int ngroups = (S + C - 1) / C;
  const T gamma = (T)st->gamma_cur;
  const int nfull = m / ROWS;  // steps where every thread holds VN valid rows
  // Few large items: an integer counter hands them out one at a time.
  if (ngroups < 8 * (int)gridDim.x) {
    for (;;) {
      if (threadIdx.x == 0) s_item = atomicAdd(&st->work_ctr, 1);
      __syncthreads();
      const int item = s_item;
      __syncthreads();
      if (item >= ngroups) break;
      const int t0 = item * C;
      const T* col[C];
  #pragma unroll
      for (int c = 0; c < C; ++c) {
        const int t = min(t0 + c, S - 1);  // a short last group repeats its last column
        col[c] = A + (size_t)sel_cols[t] * lda;
      }
      T acc[C];
  #pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = (T)0;
      const int row_t = threadIdx.x * VN;
      int step = 0;
      for (; step + U <= nfull; step += U) {
        VA a[U][C], rv[U];
  #pragma unroll
        for (int u = 0; u < U; ++u) {
          const int row = (step + u) * ROWS + row_t;
          rv[u] = *reinterpret_cast<const VA*>(r + row);
  #pragma unroll
          for (int c = 0; c < C; ++c)
            a[u][c] = NT ? __builtin_nontemporal_load(reinterpret_cast<const VA*>(col[c] + row))
                         : *reinterpret_cast<const VA*>(col[c] + row);
        }
  #pragma unroll
        for (int u = 0; u < U; ++u)
  #pragma unroll
          for (int c = 0; c < C; ++c)
  #pragma unroll
            for (int e = 0; e < VN; ++e) acc[c] += a[u][c][e] * rv[u][e];
      }
      for (; step < nfull; ++step) {
        const int row = step * ROWS + row_t;
        const VA rv = *reinterpret_cast<const VA*>(r + row);
  #pragma unroll
        for (int c = 0; c < C; ++c) {
          const VA a = NT ? __builtin_nontemporal_load(reinterpret_cast<const VA*>(col[c] + row))
                          : *reinterpret_cast<const VA*>(col[c] + row);
  #pragma unroll
          for (int e = 0; e < VN; ++e) acc[c] += a[e] * rv[e];
        }
      }
      {  // ragged tail: rows nfull*ROWS .. m-1
        const int row = nfull * ROWS + row_t;
        for (int e = 0; e < VN; ++e) {
          if (row + e < m) {
            const T rr = r[row + e];
  #pragma unroll
            for (int c = 0; c < C; ++c) acc[c] += col[c][row + e] * rr;
          }
        }
      }
  #pragma unroll
      for (int c = 0; c < C; ++c) {
        const T v = wave_sum(acc[c]);
        if (lane == 0) red[wave][c] = v;
      }
      __syncthreads();
      if (threadIdx.x < C && t0 + (int)threadIdx.x < S) {
        const int c = threadIdx.x;
        const int t = t0 + c;
        const int j = sel_cols[t];
        const T dot = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
        const T xj = x[j];
        T g = dot - (T)bp.c2 * xj;
        if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
        const T q = (T)(cn2[j] + bp.tau);
        const T xh = soft_clip<T>(xj - g / q, (T)bp.lam_eta / q, (T)bp.beta);
        const T d = gamma * (xh - xj);
        x[j] = xj + d;
        dx_sel[t] = d;
      }
    }
    return;
  }
  // Many small items (short columns): fixed round-robin assignment, the next item's column
  // indices and this item's best-response operands are loaded while the columns stream.
  int item = blockIdx.x;
  int jn[C];  // column indices of the item about to be processed
  if (item < ngroups) {
#pragma unroll
    for (int c = 0; c < C; ++c) jn[c] = sel_cols[min(item * C + c, S - 1)];
  }
  while (item < ngroups) {
    const int t0 = item * C;
    const T* col[C];
#pragma unroll
    for (int c = 0; c < C; ++c) col[c] = A + (size_t)jn[c] * lda;
    // best-response operands of this item (only threads c < C use them)
    T xj = (T)0;
    double qd = 0.0;
    int jme = 0;
    if ((int)threadIdx.x < C && t0 + (int)threadIdx.x < S) {
      jme = jn[threadIdx.x];
      xj = x[jme];
      qd = cn2[jme];
    }
    const int next = item + gridDim.x;
    T acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = (T)0;
    const int row_t = threadIdx.x * VN;
    int step = 0;
    for (; step + U <= nfull; step += U) {
      VA a[U][C], rv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int row = (step + u) * ROWS + row_t;
        rv[u] = *reinterpret_cast<const VA*>(r + row);
#pragma unroll
        for (int c = 0; c < C; ++c)
          a[u][c] = NT ? __builtin_nontemporal_load(reinterpret_cast<const VA*>(col[c] + row))
                       : *reinterpret_cast<const VA*>(col[c] + row);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int e = 0; e < VN; ++e) acc[c] += a[u][c][e] * rv[u][e];
    }
    for (; step < nfull; ++step) {
      const int row = step * ROWS + row_t;
      const VA rv = *reinterpret_cast<const VA*>(r + row);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const VA a = NT ? __builtin_nontemporal_load(reinterpret_cast<const VA*>(col[c] + row))
                        : *reinterpret_cast<const VA*>(col[c] + row);
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[c] += a[e] * rv[e];
      }
    }
    {  // ragged tail: rows nfull*ROWS .. m-1
      const int row = nfull * ROWS + row_t;
      for (int e = 0; e < VN; ++e) {
        if (row + e < m) {
          const T rr = r[row + e];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] += col[c][row + e] * rr;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const T v = wave_sum(acc[c]);
      if (lane == 0) red[wave][c] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < C && t0 + (int)threadIdx.x < S) {
      const int c = threadIdx.x;
      const int t = t0 + c;
      const T dot = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
      T g = dot - (T)bp.c2 * xj;
      if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
      const T q = (T)(qd + bp.tau);
      const T xh = soft_clip<T>(xj - g / q, (T)bp.lam_eta / q, (T)bp.beta);
      const T d = gamma * (xh - xj);
      x[jme] = xj + d;
      dx_sel[t] = d;
    }
    __syncthreads();  // red is reused by the next item
    item = next;
    if (item < ngroups) {
#pragma unroll
      for (int c = 0; c < C; ++c) jn[c] = sel_cols[min(item * C + c, S - 1)];
    }
  }
}

// Wave variant of the walk for short columns: every wave takes its own group of C
// consecutive drawn coordinates (integer work counter) and walks down them with 64 lanes x
// 16-byte loads, U row steps in flight; a butterfly per column, then lanes 0..C-1 apply
// the best response.
template <typename T, int C, int U>
__global__ void __launch_bounds__(256)
k_grad_br_wwalk(const T* __restrict__ A, long long lda, int m, const T* __restrict__ r,
                T* __restrict__ x, const double* __restrict__ cn2,
                const int* __restrict__ sel_cols, RoundState* __restrict__ st,
                T* __restrict__ dx_sel, BRParams bp) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  constexpr int ROWS = 64 * VN;
  const int lane = threadIdx.x & 63;
  const int S = st->S_cnt;
  const int ngroups = (S + C - 1) / C;
  const T gamma = (T)st->gamma_cur;
  const int nfull = m / ROWS;
  const int GR = max(1, ngroups / (int)(32 * gridDim.x));
  int item = 0, left = 0;
  for (;;) {
    if (left == 0) {
      int b = 0;
      if (lane == 0) b = atomicAdd(&st->work_ctr, GR);
      item = __shfl(b, 0, 64);
      left = GR;
    } else {
      ++item;
    }
    --left;
    if (item >= ngroups) break;
    const int t0 = item * C;
    const int cnt = min(C, S - t0);
    const T* col[C];
#pragma unroll
    for (int c = 0; c < C; ++c) col[c] = A + (size_t)sel_cols[t0 + min(c, cnt - 1)] * lda;
    T acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = (T)0;
    const int row_t = lane * VN;
    int step = 0;
    for (; step + U <= nfull; step += U) {
      VA a[U][C], rv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int row = (step + u) * ROWS + row_t;
        rv[u] = *reinterpret_cast<const VA*>(r + row);
#pragma unroll
        for (int c = 0; c < C; ++c)
          a[u][c] = __builtin_nontemporal_load(reinterpret_cast<const VA*>(col[c] + row));
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int e = 0; e < VN; ++e) acc[c] += a[u][c][e] * rv[u][e];
    }
    for (; step < nfull; ++step) {
      const int row = step * ROWS + row_t;
      const VA rv = *reinterpret_cast<const VA*>(r + row);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const VA a = __builtin_nontemporal_load(reinterpret_cast<const VA*>(col[c] + row));
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[c] += a[e] * rv[e];
      }
    }
    {
      const int row = nfull * ROWS + row_t;
      for (int e = 0; e < VN; ++e)
        if (row + e < m) {
          const T rr = r[row + e];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] += col[c][row + e] * rr;
        }
    }
    T mine = (T)0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const T v = wave_sum(acc[c]);
      if (lane == c) mine = v;
    }
    if (lane < cnt) {
      const int t = t0 + lane;
      const int j = sel_cols[t];
      const T xj = x[j];
      T g = mine - (T)bp.c2 * xj;
      if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
      const T q = (T)(cn2[j] + bp.tau);
      const T xh = soft_clip<T>(xj - g / q, (T)bp.lam_eta / q, (T)bp.beta);
      const T d = gamma * (xh - xj);
      x[j] = xj + d;
      dx_sel[t] = d;
    }
  }
}

// ------------------------------------------------------------------ fused round (dense)
// S.2-S.5 in one pass over the drawn columns, for columns that fit one 1024-thread
// workgroup: thread t owns the 16-byte row groups t, t + 1024, ..., t + (Q-1)*1024 and keeps
// those rows of r and of its workgroup's fold partial in registers.  Workgroup w takes the
// drawn coordinates [w*S/G, (w+1)*S/G) in groups of C; per group it forms the C gradients
// (wave butterflies, then the 16 wave sums in a fixed order), the best responses and the
// moves, and adds move * column into the partial from the registers that hold the column,
// so A_S is read once per round.  The next group's loads are issued before the current
// group is reduced, so one group is in flight at a time (keeping two in flight measured
// slower for 80 KB columns, and no faster for shorter ones).  Loads are never skipped
// (past the end of the share, or in a short last group, every lane reads the first 16
// bytes of A instead), which keeps the compiler's wait counts exact.
// part[w] receives workgroup w's partial (k_part_reduce adds them to r);
// st->moved_updates counts the moved coordinates.
// Longer columns (L > 0): beyond the Q row groups in registers, each thread keeps L more
// row groups of the column, of r and of its partial in LDS slots that only it touches
// (Q = the register limit, C = 1); the next column's LDS part is loaded into registers
// with the rest of the next group and stored to the slots once the current column is done.
constexpr int kFusedMaxQ32 = 5;  // row groups per thread (registers), FP32
constexpr int kFusedMaxQ64 = 3;  // and FP64
constexpr int kFusedMaxL = 3;    // row groups per thread in LDS (3 x 16 KB each for A, r, partial)
constexpr int kFusedSelCols = 4096;     // LDS list of a workgroup's share (draw in the kernel)
constexpr int kFusedSelColsL = 2048;    // the same with LDS row groups
constexpr int kFusedSelBlocks = 32768;  // blocks drawn in the kernel (32 per thread at most)

// Block draw of the fused round (on = 0: the drawn list comes from k_select).
struct FusedSel {
  const int* bp;  // block pointer (nblocks + 1)
  int nblocks;
  int on;
  uint64_t seed;
  uint64_t T;
  uint32_t inst;
  int bsz;    // > 0: every block but the last has bsz columns (the draw then reads no bp)
  int ncols;  // columns (with bsz > 0)
};

// First column and length of block i.
__device__ __forceinline__ int fs_blk_begin(const FusedSel& fs, int i) {
  return fs.bsz > 0 ? min(i * fs.bsz, fs.ncols) : fs.bp[i];
}
__device__ __forceinline__ int fs_blk_len(const FusedSel& fs, int i) {
  return fs.bsz > 0 ? min(fs.bsz, fs.ncols - i * fs.bsz) : fs.bp[i + 1] - fs.bp[i];
}

template <typename T, int Q, int C>
struct FusedBuf {
  typename V16<T>::v a[C][Q];
  int j[C];
  T x[C];
  double q2[C];
};

template <typename T, int Q, int C, int L = 0>
__global__ void __launch_bounds__(1024)
k_grad_br_fold(const T* __restrict__ A, long long lda, int m, const T* __restrict__ r,
               T* __restrict__ x, const double* __restrict__ cn2,
               const int* __restrict__ sel_cols, RoundState* __restrict__ st,
               T* __restrict__ part, long long ldp, BRParams bp, FusedSel fs) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  constexpr int LL = L > 0 ? L : 1;
  static_assert(L == 0 || C == 1, "LDS row groups go with one column per group");
  __shared__ T red[2][C][16];
  __shared__ int s_scan[17];
  __shared__ int s_cols[L > 0 ? kFusedSelColsL : kFusedSelCols];
  // thread-private LDS row groups: the current column, r, the partial
  __shared__ VA s_ext[L > 0 ? 3 * L * 1024 : 1];
  VA* s_a = s_ext;
  VA* s_rr = s_ext + LL * 1024;
  VA* s_pa = s_ext + 2 * LL * 1024;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int G = gridDim.x;
  const int nq = (m + VN - 1) / VN;  // row groups holding rows < m (lda covers them)
  // Byte offsets of the owned row groups within a column (register slots q < Q, then LDS
  // slots Q + l).  The last slot is the only one that can reach past row m: it is clamped
  // to the last row group, and its rows >= m are zeroed after each load (A's padding rows
  // may hold anything).
  constexpr int QL = Q + L;
  uint32_t boff[Q], loff[LL];
#pragma unroll
  for (int q = 0; q < Q; ++q) boff[q] = (uint32_t)((q * 1024 + tid) * 16);
#pragma unroll
  for (int l = 0; l < LL; ++l) loff[l] = (uint32_t)(((Q + l) * 1024 + tid) * 16);
  if (L == 0)
    boff[Q - 1] = (uint32_t)(min((Q - 1) * 1024 + tid, nq - 1) * 16);
  else
    loff[LL - 1] = (uint32_t)(min((QL - 1) * 1024 + tid, nq - 1) * 16);
  const int rlast = ((QL - 1) * 1024 + tid) * VN;
  const int nlast = max(0, min(VN, m - rlast));  // valid rows of the last slot
  VA rr[Q], pa[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int row = (q * 1024 + tid) * VN;
    if (row + VN <= m) {
      rr[q] = *reinterpret_cast<const VA*>(r + row);
    } else {
#pragma unroll
      for (int e = 0; e < VN; ++e) rr[q][e] = row + e < m ? r[row + e] : (T)0;
    }
#pragma unroll
    for (int e = 0; e < VN; ++e) pa[q][e] = (T)0;
  }
  if constexpr (L > 0) {
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int row = ((Q + l) * 1024 + tid) * VN;
      VA v;
      if (row + VN <= m) {
        v = *reinterpret_cast<const VA*>(r + row);
      } else {
#pragma unroll
        for (int e = 0; e < VN; ++e) v[e] = row + e < m ? r[row + e] : (T)0;
      }
      s_rr[l * 1024 + tid] = v;
#pragma unroll
      for (int e = 0; e < VN; ++e) v[e] = (T)0;
      s_pa[l * 1024 + tid] = v;
    }
  }
  // S.1, here or in k_select.  Here (fs.on): every workgroup evaluates the draw of every
  // block (the k_select draw, round st->k), scans the drawn columns in block order and lists
  // its own share [t0, t1) in LDS; the round state is advanced afterwards by k_part_reduce,
  // so this round's step is st->gamma_next.
  int S;
  T gamma;
  if (fs.on) {
    const long long k = st->k;
    gamma = (T)st->gamma_next;
    const int per = (fs.nblocks + 1023) / 1024;  // <= 32 (host check)
    const int b0 = min(fs.nblocks, tid * per), b1 = min(fs.nblocks, b0 + per);
    int cnt = 0;
    uint32_t mask = 0;
    for (int i = b0; i < b1; ++i) {
      if (block_drawn((uint32_t)i, (uint64_t)k, fs.inst, fs.seed, fs.T)) {
        cnt += fs_blk_len(fs, i);
        mask |= 1u << (i - b0);
      }
    }
    int off = block_exclusive_scan_1024(cnt, s_scan, &S);
    const int u0 = (int)((long long)S * blockIdx.x / G);
    const int u1 = (int)((long long)S * (blockIdx.x + 1) / G);
    for (int i = b0; i < b1; ++i) {
      if (mask & (1u << (i - b0))) {
        const int c0 = fs_blk_begin(fs, i), len = fs_blk_len(fs, i);
        const int lo = max(off, u0), hi = min(off + len, u1);
        for (int t = lo; t < hi; ++t) s_cols[t - u0] = c0 + (t - off);
        off += len;
      }
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid == 0) st->S_cnt = S;
  } else {
    S = st->S_cnt;
    gamma = (T)st->gamma_cur;
  }
  const int t0 = (int)((long long)S * blockIdx.x / G);
  const int t1 = (int)((long long)S * (blockIdx.x + 1) / G);
  const int nitems = (t1 - t0 + C - 1) / C;
  long long moved = 0;
  VA aln[LL];  // the LDS part of the next column, staged in registers
  auto load = [&](int tb, FusedBuf<T, Q, C>& B) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const bool ok = tb + c < t1;  // uniform
      const uint32_t omask = ok ? 0xffffffffu : 0u;
      B.j[c] = ok ? (fs.on ? s_cols[tb + c - t0] : sel_cols[tb + c]) : 0;
      const char* col = reinterpret_cast<const char*>(A + (size_t)B.j[c] * lda);
#pragma unroll
      for (int q = 0; q < Q; ++q)
        B.a[c][q] = __builtin_nontemporal_load(
            reinterpret_cast<const VA*>(col + (boff[q] & omask)));
      if constexpr (L > 0) {
#pragma unroll
        for (int l = 0; l < L; ++l)
          aln[l] = __builtin_nontemporal_load(
              reinterpret_cast<const VA*>(col + (loff[l] & omask)));
      }
      B.x[c] = x[B.j[c]];
      B.q2[c] = cn2[B.j[c]];
    }
  };
  // the staged LDS part becomes the current column's (rows >= m zeroed)
  auto stage = [&]() {
    if constexpr (L > 0) {
#pragma unroll
      for (int l = 0; l < L; ++l) {
        VA v = aln[l];
        if (l == L - 1 && nlast < VN) {
#pragma unroll
          for (int e = 0; e < VN; ++e) v[e] = e < nlast ? v[e] : (T)0;
        }
        s_a[l * 1024 + tid] = v;
      }
    }
  };
  auto process = [&](int tb, FusedBuf<T, Q, C>& B, int buf) {
    T acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (L == 0 && nlast < VN) {
#pragma unroll
        for (int e = 0; e < VN; ++e) B.a[c][Q - 1][e] = e < nlast ? B.a[c][Q - 1][e] : (T)0;
      }
      acc[c] = (T)0;
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[c] += B.a[c][q][e] * rr[q][e];
      if constexpr (L > 0) {
#pragma unroll
        for (int l = 0; l < L; ++l) {
          const VA av = s_a[l * 1024 + tid], rv = s_rr[l * 1024 + tid];
#pragma unroll
          for (int e = 0; e < VN; ++e) acc[c] += av[e] * rv[e];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const T v = wave_sum(acc[c]);
      if (lane == 0) red[buf][c][wave] = v;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (tb + c < t1) {
        const T* rs = red[buf][c];
        const T dot = (((rs[0] + rs[1]) + (rs[2] + rs[3])) + ((rs[4] + rs[5]) + (rs[6] + rs[7]))) +
                      (((rs[8] + rs[9]) + (rs[10] + rs[11])) +
                       ((rs[12] + rs[13]) + (rs[14] + rs[15])));
        const T xj = B.x[c];
        T g = dot - (T)bp.c2 * xj;
        if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
        const T qq = (T)(B.q2[c] + bp.tau);
        const T xh = soft_clip<T>(xj - g / qq, (T)bp.lam_eta / qq, (T)bp.beta);
        const T d = gamma * (xh - xj);
        if (d != (T)0) {
#pragma unroll
          for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int e = 0; e < VN; ++e) pa[q][e] += B.a[c][q][e] * d;
          if constexpr (L > 0) {
#pragma unroll
            for (int l = 0; l < L; ++l) {
              const VA av = s_a[l * 1024 + tid];
              VA pv = s_pa[l * 1024 + tid];
#pragma unroll
              for (int e = 0; e < VN; ++e) pv[e] += av[e] * d;
              s_pa[l * 1024 + tid] = pv;
            }
          }
          ++moved;
        }
        if (tid == 0) x[B.j[c]] = xj + d;
      }
    }
  };
  if (nitems > 0) {
    FusedBuf<T, Q, C> B0, B1;
    load(t0, B0);
    stage();
    for (int it = 0; it < nitems; ++it) {
      load(t0 + (it + 1) * C, B1);
      process(t0 + it * C, B0, it & 1);
      B0 = B1;
      stage();
    }
  }
  T* dst = part + (size_t)blockIdx.x * ldp;
  if constexpr (L == 0) {
#pragma unroll
    for (int q = 0; q < Q - 1; ++q)
      *reinterpret_cast<VA*>(dst + (q * 1024 + tid) * VN) = pa[q];
    if ((Q - 1) * 1024 + tid < nq) *reinterpret_cast<VA*>(dst + rlast) = pa[Q - 1];
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q)
      *reinterpret_cast<VA*>(dst + (q * 1024 + tid) * VN) = pa[q];
#pragma unroll
    for (int l = 0; l < L - 1; ++l)
      *reinterpret_cast<VA*>(dst + ((Q + l) * 1024 + tid) * VN) = s_pa[l * 1024 + tid];
    if ((QL - 1) * 1024 + tid < nq)
      *reinterpret_cast<VA*>(dst + rlast) = s_pa[(L - 1) * 1024 + tid];
  }
  if (tid == 0) {
    if (moved) atomicAdd(reinterpret_cast<unsigned long long*>(&st->moved_updates),
                         (unsigned long long)moved);
    if (blockIdx.x == 0) st->ngroups = G;
  }
}

// r[i] = base[i] + sum over w < G of part[w][i] (base may be r).  A 256-thread workgroup
// takes 16 row groups of 16 bytes; lane group v (16 lanes, one per row group) adds the
// partials [v*G/16, (v+1)*G/16) in order, then one thread per row group adds the 16 group
// sums to base in group order (the same order for any grid).
// With advance != 0 (the block draw ran inside the fused kernel) it also advances the round
// state the way k_select does: next round, step, drawn-coordinate total.
constexpr int kPartRows = 16;  // row groups per workgroup of k_part_reduce
template <typename T>
__global__ void __launch_bounds__(256)
k_part_reduce(const T* __restrict__ part, long long ldp, int G, int m, const T* base, T* r,
              RoundState* __restrict__ st, int advance) {
  if (advance && blockIdx.x == 0 && threadIdx.x == 0) {
    const double g = st->gamma_next;
    st->coord_updates += st->S_cnt;
    st->work_ctr = 0;
    st->k += 1;
    st->gamma_cur = g;
    st->gamma_next = g * (1.0 - st->gamma_mu * g);
  }
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  constexpr int KMAX = 16;  // partials per lane group (G <= 256)
  __shared__ VA sh[16][kPartRows];
  const int rg = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int row = (blockIdx.x * kPartRows + rg) * VN;
  VA acc;
#pragma unroll
  for (int e = 0; e < VN; ++e) acc[e] = (T)0;
  const int g0 = grp * G / 16, g1 = (grp + 1) * G / 16;
  if (row < m && g1 > g0) {
    VA v[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      v[k] = *reinterpret_cast<const VA*>(part + (size_t)min(g0 + k, g1 - 1) * ldp + row);
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (g0 + k < g1) acc += v[k];
  }
  sh[grp][rg] = acc;
  __syncthreads();
  if (grp == 0 && row < m) {
    if (row + VN <= m) {
      VA s = *reinterpret_cast<const VA*>(base + row);
#pragma unroll
      for (int w = 0; w < 16; ++w) s += sh[w][rg];
      *reinterpret_cast<VA*>(r + row) = s;
    } else {
      for (int e = 0; e < m - row; ++e) {
        T s = base[row + e];
#pragma unroll
        for (int w = 0; w < 16; ++w) s += sh[w][rg][e];
        r[row + e] = s;
      }
    }
  }
}

// ------------------------------------------------------------------ compaction
// Two passes over v[0..N): per-chunk nonzero counts, then an ordered scatter of
// (index, value) for the nonzero entries.  N is read from device memory.
template <typename T>
__global__ void __launch_bounds__(1024) k_compact_count(const T* __restrict__ v,
                                                        const int* __restrict__ N_ptr,
                                                        int* __restrict__ chunk_cnt) {
  __shared__ int sh[16];
  const int N = *N_ptr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = blockIdx.x; c * kChunk < N; c += gridDim.x) {
    const int t = c * kChunk + threadIdx.x;
    const bool nz = t < N && v[t] != (T)0;
    const uint64_t bal = __ballot(nz);
    if (lane == 0) sh[wave] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
      int s = 0;
      for (int w = 0; w < 16; ++w) s += sh[w];
      chunk_cnt[c] = s;
    }
    __syncthreads();
  }
}

// Writes list entries in ascending position; the workgroup that owns the last chunk
// stores the count and the fold's column grouping (G entries per group, <= kMaxGroups).
template <typename T>
__global__ void __launch_bounds__(1024)
k_compact_scatter(const T* __restrict__ v, const int* __restrict__ idx,
                  const int* __restrict__ N_ptr, const int* __restrict__ chunk_cnt,
                  int* __restrict__ J_idx, T* __restrict__ J_val, RoundState* __restrict__ st,
                  int count_moved) {
  __shared__ int sh[17];
  __shared__ int sh_base;
  const int N = *N_ptr;
  const int nch = (N + kChunk - 1) / kChunk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (N == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    st->J_cnt = 0;
    st->G = 1;
    st->ngroups = 0;
  }
  for (int c = blockIdx.x; c < nch; c += gridDim.x) {
    // base = sum of the counts of the chunks before c (fixed order)
    int part = 0;
    for (int q = threadIdx.x; q < c; q += 1024) part += chunk_cnt[q];
    int tot;
    (void)block_exclusive_scan_1024(part, sh, &tot);
    if (threadIdx.x == 0) sh_base = tot;
    __syncthreads();
    const int base = sh_base;
    const int t = c * kChunk + threadIdx.x;
    const bool nz = t < N && v[t] != (T)0;
    const uint64_t bal = __ballot(nz);
    if (lane == 0) sh[wave] = __popcll(bal);
    __syncthreads();
    int woff = 0, ctot = 0;
    for (int w = 0; w < 16; ++w) {
      const int s = sh[w];
      if (w < wave) woff += s;
      ctot += s;
    }
    if (nz) {
      const int pos = base + woff + lanes_below(bal);
      J_idx[pos] = idx ? idx[t] : t;
      J_val[pos] = v[t];
    }
    if (c == nch - 1 && threadIdx.x == 0) {
      const int J = base + ctot;
      int G = (J + kMaxGroups - 1) / kMaxGroups;
      if (G < 16) G = 16;
      st->J_cnt = J;
      if (count_moved) st->moved_updates += J;
      st->G = G;
      st->ngroups = (J + G - 1) / G;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ residual fold
// part[g][i] = sum over list entries e of group g (ascending) of A[i, J_idx[e]] * J_val[e].
// Tile = (256*VN rows) x (one group); 16-byte loads down each listed column.
template <typename T, typename Acc>
__global__ void __launch_bounds__(256)
k_fold_partial(const T* __restrict__ A, long long lda, int m, const int* __restrict__ J_idx,
               const T* __restrict__ J_val, const RoundState* __restrict__ st,
               Acc* __restrict__ part, long long ldp) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  const int J = st->J_cnt, G = st->G, ng = st->ngroups;
  const int rows_tile = 256 * VN;
  const int nrt = (m + rows_tile - 1) / rows_tile;
  for (int tile = blockIdx.x; tile < nrt * ng; tile += gridDim.x) {
    const int g = tile / nrt, rt = tile - g * nrt;
    const int e0 = g * G, e1 = min(J, e0 + G);
    const int row0 = rt * rows_tile + threadIdx.x * VN;
    Acc acc[VN];
#pragma unroll
    for (int v = 0; v < VN; ++v) acc[v] = (Acc)0;
    if (row0 + VN <= m) {
      int e = e0;
      for (; e + 4 <= e1; e += 4) {
        VA a[4];
        Acc d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = J_idx[e + u];
          d[u] = (Acc)J_val[e + u];
          a[u] = __builtin_nontemporal_load(
              reinterpret_cast<const VA*>(A + (size_t)j * lda + row0));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < VN; ++v) acc[v] += (Acc)a[u][v] * d[u];
      }
      for (; e < e1; ++e) {
        const int j = J_idx[e];
        const Acc d = (Acc)J_val[e];
        const VA a = __builtin_nontemporal_load(
            reinterpret_cast<const VA*>(A + (size_t)j * lda + row0));
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[v] += (Acc)a[v] * d;
      }
    } else if (row0 < m) {
      for (int e = e0; e < e1; ++e) {
        const int j = J_idx[e];
        const Acc d = (Acc)J_val[e];
        for (int v = 0; v < m - row0; ++v) acc[v] += (Acc)A[(size_t)j * lda + row0 + v] * d;
      }
    }
    if (row0 < m) {
      Acc* dst = part + (size_t)g * ldp + row0;
#pragma unroll
      for (int v = 0; v < VN; ++v)
        if (row0 + v < m) dst[v] = acc[v];
    }
  }
}

// out[i] = base_scale*base[i] + sum_{g ascending} part[g][i]  (also to out64 when given)
template <typename TB, typename Acc, typename TO>
__global__ void __launch_bounds__(256)
k_fold_reduce(const TB* __restrict__ base, double base_scale, const Acc* __restrict__ part,
              long long ldp, const RoundState* __restrict__ st, int m, TO* __restrict__ out,
              double* __restrict__ out64) {
  const int ng = st->ngroups;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    Acc s = (Acc)(base_scale * (double)base[i]);
#pragma unroll 8
    for (int g = 0; g < ng; ++g) s += part[(size_t)g * ldp + i];
    if (out) out[i] = (TO)s;
    if (out64) out64[i] = (double)s;
  }
}

// ------------------------------------------------------------------ FP64 checks
// Deterministic block reduction of three doubles (256 threads).
__device__ __forceinline__ void block_sum3_256(double a, double b, double c, double* dst) {
  __shared__ double sh[3][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if (lane == 0) {
    sh[0][wave] = a;
    sh[1][wave] = b;
    sh[2][wave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < 3; ++q) dst[q] = ((sh[q][0] + sh[q][1]) + sh[q][2]) + sh[q][3];
  }
}

// part[3*blk + {0,1,2}] = (sum r_i^2, sum x_j^2, sum h(x_j)) over this block's share.
template <typename TX, typename TR>
__global__ void __launch_bounds__(256) k_obj_partial(const TR* __restrict__ r, int m,
                                                     const TX* __restrict__ x, int n,
                                                     BRParams bp, double* __restrict__ part) {
  double sr = 0.0, sx = 0.0, sh = 0.0;
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const double v = (double)r[i];
    sr += v * v;
  }
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
    const double v = (double)x[j];
    sx += v * v;
    sh += h_value<double>(v, bp);
  }
  block_sum3_256(sr, sx, sh, part + 3 * blockIdx.x);
}

// out[0] = F = 1/2 sum r^2 - c sum x^2 + lam sum h(x); out[1..3] = the three sums.
// 256 threads: thread i sums parts i, i+256, ... in order, then a fixed-order tree.
static __global__ void __launch_bounds__(256) k_obj_final(const double* __restrict__ part,
                                                          int nparts, double c, double lam,
                                                          double* __restrict__ out) {
  double sr = 0.0, sx = 0.0, sh = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256) {
    sr += part[3 * b];
    sx += part[3 * b + 1];
    sh += part[3 * b + 2];
  }
  __shared__ double res[3];
  block_sum3_256(sr, sx, sh, res);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = 0.5 * res[0] - c * res[1] + lam * res[2];
    out[1] = res[0];
    out[2] = res[1];
    out[3] = res[2];
  }
}

// Stationarity probe over every coordinate with an FP64 residual: per wave the max of
// |xh_j - x_j|, the sum of (x_j - y_j)^2 with y the unit-step prox point (M_F) and the
// count of xh_j != 0.
template <typename T>
__global__ void __launch_bounds__(256)
k_probe(const T* __restrict__ A, long long lda, int m, const double* __restrict__ r64,
        const T* __restrict__ x, int n, const double* __restrict__ cn2, BRParams bp,
        double* __restrict__ wmax, double* __restrict__ wsum, int* __restrict__ wcnt) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nw = gridDim.x * 4;
  double mx = 0.0, sm = 0.0;
  int cnt = 0;
  for (int j = gw; j < n; j += nw) {
    const double dot = col_dot<T, double, double, 4>(A + (size_t)j * lda, r64, m, lane);
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
  if (lane == 0) {
    wmax[gw] = mx;
    wsum[gw] = sm;
    wcnt[gw] = cnt;
  }
}

// out[0] = max, out[1] = sqrt(sum), out[2] = count (fixed summation order, 256 threads).
static __global__ void __launch_bounds__(256) k_probe_final(const double* __restrict__ wmax,
                                                            const double* __restrict__ wsum,
                                                            const int* __restrict__ wcnt, int nw,
                                                            double* __restrict__ out) {
  double mx = 0.0, sm = 0.0, cnt = 0.0;
  for (int w = threadIdx.x; w < nw; w += 256) {
    mx = fmax(mx, wmax[w]);
    sm += wsum[w];
    cnt += (double)wcnt[w];
  }
  __shared__ double shm[4];
  __shared__ double res[3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double wm = wave_max(mx);
  if (lane == 0) shm[wave] = wm;
  block_sum3_256(sm, cnt, 0.0, res);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = fmax(fmax(shm[0], shm[1]), fmax(shm[2], shm[3]));
    out[1] = sqrt(res[0]);
    out[2] = res[1];
  }
}

}  // namespace sca
