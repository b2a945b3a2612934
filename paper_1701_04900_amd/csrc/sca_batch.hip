// Batched engine of libsca: many dense instances of uneven size run as one block-diagonal
// problem.  A device descriptor table holds each instance's A (borrowed), sizes, offsets
// into the concatenated x / r / b, lambda, c, beta, tau, F* and its Philox instance word.
// Per round the drawn blocks of every active instance, the gradient work items (<= C
// columns of one block), the moved-coordinate list and the fold tiles are all built on the
// device; convergence flags are updated on the device, so a graph of E rounds plus a
// check is replayed without host decisions in between.  Instance k follows exactly the
// trajectory of the plain path run with instance word k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <vector>

#include "sca_batch_internal.h"

using namespace sca;

namespace {


__device__ __forceinline__ int upper_idx(const int* __restrict__ off, int K, int v) {
  // largest k in [0, K) with off[k] <= v (off ascending, off[0] = 0)
  int lo = 0, hi = K - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= v)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ S.1 over all instances
// Cost of one drawn column in the split of the fused round's work: its rows plus a fixed
// part for the per-column work that does not scale with m (the group's barriers and best
// responses, which dominate at these column lengths).  On 256 instances with m in [500, 8000]
// the batched solve takes 14.05 / 13.71 / 13.19 / 12.90 / 13.05 s with 512 / 1024 / 4096 /
// 16384 / 65536.
constexpr int kBFColCost = 16384;

__global__ void __launch_bounds__(1024)
k_bsel_count(int Btot, const int* __restrict__ blk_inst, const int* __restrict__ blk_len,
             const BInst* __restrict__ inst, const int* __restrict__ active, uint64_t seed,
             uint64_t T, const BState* __restrict__ st, int* __restrict__ blk_cols,
             int* __restrict__ chunk_cols, int* __restrict__ chunk_items,
             long long* __restrict__ chunk_cost, int* __restrict__ inst_lo,
             int* __restrict__ inst_hi, long long* __restrict__ inst_upd) {
  __shared__ int sh[2][16];
  __shared__ long long shc[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long k = st->rs.k;
  for (int c = blockIdx.x; c * kChunk < Btot; c += gridDim.x) {
    const int b = c * kChunk + threadIdx.x;
    int cols = 0, items = 0;
    long long cost = 0;
    if (b < Btot) {
      const int q = blk_inst[b];
      if (b == inst[q].blk_off) {  // every instance's first block resets its item range
        inst_lo[q] = 0x7fffffff;
        inst_hi[q] = -1;
      }
      if (active[q] &&
          block_drawn((uint32_t)(b - inst[q].blk_off), (uint64_t)k, inst[q].inst_id, seed, T)) {
        cols = blk_len[b];
        items = (cols + kBC - 1) / kBC;
        cost = (long long)cols * (inst[q].m + kBFColCost);
        atomicAdd((unsigned long long*)&inst_upd[q], (unsigned long long)cols);
      }
      blk_cols[b] = cols;
    }
    const int wc = wave_sum(cols), wi = wave_sum(items);
    const long long wk = wave_sum_i64(cost);
    if (lane == 0) {
      sh[0][wave] = wc;
      sh[1][wave] = wi;
      shc[wave] = wk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int a = 0, i = 0;
      long long cc = 0;
      for (int w = 0; w < 16; ++w) {
        a += sh[0][w];
        i += sh[1][w];
        cc += shc[w];
      }
      chunk_cols[c] = a;
      chunk_items[c] = i;
      chunk_cost[c] = cc;
    }
    __syncthreads();
  }
}

// Exclusive scan of 64-bit values over a 1024-thread block; 'sh' needs 17 entries.
__device__ __forceinline__ long long block_exclusive_scan_1024_i64(long long v, long long* sh,
                                                                   long long* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long long inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const long long t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long run = 0;
    for (int w = 0; w < 16; ++w) {
      const long long t = sh[w];
      sh[w] = run;
      run += t;
    }
    sh[16] = run;
  }
  __syncthreads();
  const long long res = sh[wave] + inc - v;
  *total = sh[16];
  __syncthreads();
  return res;
}

// Ordered lists of the round: drawn columns and work items (<= kBC columns of one block).
// For the fused round (G > 0) also the cost prefix of every item, the first item of every
// workgroup's share -- workgroup w takes the items whose cost prefix p satisfies
// floor(p G / T) = w (T = the round's total cost), i.e. wg_first[w] is the first item with
// p >= ceil(w T / G) -- and each instance's first and last item.
__global__ void __launch_bounds__(1024)
k_bsel_scatter(int Btot, const int* __restrict__ blk_inst, const int* __restrict__ blk_col0,
               const int* __restrict__ blk_cols, const int* __restrict__ chunk_cols,
               const int* __restrict__ chunk_items, const long long* __restrict__ chunk_cost,
               const BInst* __restrict__ inst, BState* __restrict__ st,
               int* __restrict__ sel_cols, BItem* __restrict__ items,
               long long* __restrict__ item_pref, int* __restrict__ wg_first, int G,
               int* __restrict__ inst_lo, int* __restrict__ inst_hi) {
  __shared__ int sh[17];
  __shared__ long long shl[17];
  __shared__ int s_base[2];
  __shared__ long long s_cbase[2];
  const int nch = (Btot + kChunk - 1) / kChunk;
  for (int c = blockIdx.x; c < nch; c += gridDim.x) {
    int pc = 0, pi = 0;
    long long pk = 0, pall = 0;
    for (int q = threadIdx.x; q < nch; q += 1024) {
      if (q < c) {
        pc += chunk_cols[q];
        pi += chunk_items[q];
        pk += chunk_cost[q];
      }
      pall += chunk_cost[q];
    }
    int tc, ti;
    long long tk, tall;
    (void)block_exclusive_scan_1024(pc, sh, &tc);
    (void)block_exclusive_scan_1024(pi, sh, &ti);
    (void)block_exclusive_scan_1024_i64(pk, shl, &tk);
    (void)block_exclusive_scan_1024_i64(pall, shl, &tall);
    if (threadIdx.x == 0) {
      s_base[0] = tc;
      s_base[1] = ti;
      s_cbase[0] = tk;
      s_cbase[1] = tall;
    }
    __syncthreads();
    const long long Tc = s_cbase[1];
    const int b = c * kChunk + threadIdx.x;
    const int cols = b < Btot ? blk_cols[b] : 0;
    const int nit = (cols + kBC - 1) / kBC;
    const int q = b < Btot ? blk_inst[b] : 0;
    const long long per = cols ? (long long)(inst[q].m + kBFColCost) : 0;
    int totc, toti;
    long long totk;
    const int oc = s_base[0] + block_exclusive_scan_1024(cols, sh, &totc);
    const int oi = s_base[1] + block_exclusive_scan_1024(nit, sh, &toti);
    const long long ok = s_cbase[0] + block_exclusive_scan_1024_i64(cols * per, shl, &totk);
    if (cols) {
      const int c0 = blk_col0[b];
      for (int u = 0; u < cols; ++u) sel_cols[oc + u] = c0 + u;
      for (int u = 0; u < nit; ++u) {
        BItem it;
        it.pos = oc + u * kBC;
        it.cnt = min(kBC, cols - u * kBC);
        it.inst = q;
        items[oi + u] = it;
        if (G > 0) {
          const long long p = ok + (long long)u * kBC * per;
          const long long e = p + it.cnt * per;
          item_pref[oi + u] = p;
          // the workgroups whose share starts right after this item
          const long long w0 = p * G / Tc + 1, w1 = e * G / Tc;
          for (long long w = w0; w <= w1; ++w) wg_first[w] = oi + u + 1;
          if (oi + u == 0) wg_first[0] = 0;
        }
      }
      if (G > 0) {
        atomicMin(&inst_lo[q], oi);
        atomicMax(&inst_hi[q], oi + nit - 1);
      }
    }
    if (c == nch - 1 && threadIdx.x == 0) {
      st->rs.S_cnt = s_base[0] + totc;
      st->items = s_base[1] + toti;
      st->cost = Tc;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (Btot == 0) {
      st->rs.S_cnt = 0;
      st->items = 0;
      st->cost = 0;
    }
    st->rs.work_ctr = 0;
    st->rs.k += 1;
    const double g = st->rs.gamma_next;
    st->rs.gamma_cur = g;
    st->rs.gamma_next = g * (1.0 - st->rs.gamma_mu * g);
  }
}

// ------------------------------------------------------------------ S.2 + S.4
// The workgroup walk of the plain path, one work item (<= kBC columns of one block) at a time.
template <typename T, int U>
__global__ void __launch_bounds__(256)
k_bgrad(const BInst* __restrict__ inst, const BItem* __restrict__ items,
        const int* __restrict__ sel_cols, const T* __restrict__ r_all, T* __restrict__ x_all,
        const double* __restrict__ cn2, BState* __restrict__ st, T* __restrict__ dx_sel,
        BRParams bp0) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  constexpr int ROWS = 256 * VN;
  constexpr int C = kBC;
  __shared__ T red[4][C];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nitems = st->items;
  const T gamma = (T)st->rs.gamma_cur;
  const int GR = max(1, nitems / (int)(8 * gridDim.x));  // items taken per counter update
  int item = 0, left = 0;
  for (;;) {
    if (left == 0) {
      if (threadIdx.x == 0) s_item = atomicAdd(&st->rs.work_ctr, GR);
      __syncthreads();
      item = s_item;
      left = GR;
      __syncthreads();
    } else {
      ++item;
    }
    --left;
    if (item >= nitems) break;
    const BItem it = items[item];
    const BInst& I = inst[it.inst];
    const T* A = (const T*)I.A;
    const int m = I.m;
    const T* r = r_all + I.row_off;
    const T* col[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = it.pos + min(c, it.cnt - 1);
      col[c] = A + (size_t)(sel_cols[t] - I.col_off) * I.lda;
    }
    T acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = (T)0;
    const int nfull = m / ROWS;
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
    if ((int)threadIdx.x < it.cnt) {
      const int c = threadIdx.x;
      const int t = it.pos + c;
      const int j = sel_cols[t];
      BRParams bp = bp0;
      bp.tau = I.tau;
      bp.lam = I.lam;
      bp.lam_eta = I.lam * bp0.eta;
      bp.c2 = 2.0 * I.c;
      bp.beta = I.beta;
      const T dot = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
      const T xj = x_all[j];
      T g = dot - (T)bp.c2 * xj;
      if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
      const T q = (T)(cn2[j] + bp.tau);
      const T xh = soft_clip<T>(xj - g / q, (T)bp.lam_eta / q, (T)bp.beta);
      const T d = gamma * (xh - xj);
      x_all[j] = xj + d;
      dx_sel[t] = d;
    }
  }
}

// ------------------------------------------------------------------ fused round
// S.2-S.5 of every drawn column of every instance in one pass: a 512-thread workgroup holds
// a group of columns of one instance in registers -- thread t owns the 16-byte row groups
// t, t + 512, ..., t + (Q-1)*512 of each, Q = the instance's row groups per thread (1, 2 or
// 4), C = bf_cols(Q) columns per group (128 bytes per thread for Q <= 2, 64 for Q = 4) --
// with the same rows of the instance's r and of its own fold partial.  Workgroup w takes a
// contiguous share of the round's items (the shares are cut by cost, rows plus a fixed part
// per column, see k_bsel_scatter), so every partial sum has a fixed order.  When its share
// moves on to the next instance, the workgroup writes its partial: straight into r when it
// held all of that instance's items this round, otherwise into slot (w + k) for
// k_bfused_reduce.  Row groups beyond an instance's m are clamped to its last one and their
// values masked (A's padding rows may hold anything).  Registers are kept to 128 per thread
// so that two workgroups share a compute unit: their groups in flight hide each other's
// load latency (one workgroup with a prefetched second group measured slower).
constexpr int kBFThreads = 512;
constexpr int kBFWaves = kBFThreads / 64;
constexpr int kBFMaxQ = 4;        // FP32 m <= 8192, FP64 m <= 4096
constexpr int kBFMaxWgPerCu = 4;  // the partial slots are allocated for this many
constexpr int kBFSlots = 4;       // the grad_cols value of this kernel's launch shape
// Columns per group for Q row groups of 16 bytes per thread: 8 (Q = 1), 4 (Q = 2), 1 (Q = 4),
// so that a group is 128 bytes per thread where Q <= 2 (64 bytes for Q = 4: a larger group
// there exceeds the 128 registers of two workgroups per CU).  Against 4/Q columns (64 bytes
// for every Q), the batched solve of 256 instances with m in [500, 8000]: 15.1 -> 14.0 s
// (6 registers of the FP32 kernel spill; 6 columns for Q = 1: 16.5 s; 2 columns for Q = 4:
// 14.4 s).
constexpr int bf_cols(int Q) { return Q == 1 ? 8 : Q == 2 ? 4 : 1; }
constexpr int kBFMaxC = bf_cols(1);

__device__ __forceinline__ int bf_wg_of(long long pref, long long Tc, int G) {
  return (int)min((long long)(G - 1), pref * G / Tc);
}

// Row groups per thread for an instance of nq 16-byte row groups.
__device__ __forceinline__ int bf_q_of(int nq) {
  return nq <= kBFThreads ? 1 : nq <= 2 * kBFThreads ? 2 : 4;
}

// One group of C = bf_cols(Q) consecutive columns j0 .. j0+cnt-1 of instance I: the
// columns' row groups (masked past m), the C dot products with r (wave sums, then the 8
// wave sums in a fixed order), the best responses and moves (threads c < cnt, broadcast
// through LDS) and the fold into this thread's rows of the partial.
template <typename T, int Q>
__device__ __forceinline__ void bf_group(const BInst& I, int nq, int j0, int cnt,
                                         typename V16<T>::v (&rr)[kBFMaxQ],
                                         typename V16<T>::v (&pa)[kBFMaxQ],
                                         const int (&nv)[kBFMaxQ], T (*red)[kBFWaves],
                                         T* s_d,
                                         int lane, int wave, int tid, T gamma,
                                         const BRParams& bp, T* __restrict__ x_all,
                                         const double* __restrict__ cn2, long long& moved) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  constexpr int C = bf_cols(Q);
  const char* A = reinterpret_cast<const char*>(I.A);
  // the best-response inputs of column tid (threads < cnt) are loaded with the column
  T xj = (T)0;
  double q2 = 0.0;
  if (tid < cnt) {
    xj = x_all[j0 + tid];
    q2 = cn2[j0 + tid];
  }
  VA a[C][Q];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const char* col = A + (size_t)(j0 + min(c, cnt - 1) - I.col_off) * I.lda * sizeof(T);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int gi = min(q * kBFThreads + tid, nq - 1);
      a[c][q] = __builtin_nontemporal_load(reinterpret_cast<const VA*>(col + (size_t)gi * 16));
    }
  }
  T acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int e = 0; e < VN; ++e) a[c][q][e] = e < nv[q] ? a[c][q][e] : (T)0;
    acc[c] = (T)0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int e = 0; e < VN; ++e) acc[c] += a[c][q][e] * rr[q][e];
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const T v = wave_sum(acc[c]);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (tid < cnt) {
    const T* rs = red[tid];
    const T dot = ((rs[0] + rs[1]) + (rs[2] + rs[3])) + ((rs[4] + rs[5]) + (rs[6] + rs[7]));
    T g = dot - (T)bp.c2 * xj;
    if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
    const T qq = (T)(q2 + I.tau);
    const T xh = soft_clip<T>(xj - g / qq, (T)bp.lam_eta / qq, (T)bp.beta);
    const T d = gamma * (xh - xj);
    x_all[j0 + tid] = xj + d;
    s_d[tid] = d;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const T d = c < cnt ? s_d[c] : (T)0;
    if (d != (T)0) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < VN; ++e) pa[q][e] += a[c][q][e] * d;
      if (tid == 0) ++moved;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBFThreads, 4)  // 4 waves per SIMD: two workgroups per CU
k_bfused(const BInst* __restrict__ inst, const BItem* __restrict__ items,
         const long long* __restrict__ item_pref, const int* __restrict__ wg_first,
         const int* __restrict__ inst_lo, const int* __restrict__ inst_hi,
         const int* __restrict__ sel_cols, T* __restrict__ r_all, T* __restrict__ x_all,
         const double* __restrict__ cn2, BState* __restrict__ st, T* __restrict__ part,
         long long pst, BRParams bp0) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  __shared__ T red[kBFMaxC][kBFWaves];
  __shared__ T s_d[kBFMaxC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int G = gridDim.x, w = blockIdx.x;
  if (st->items == 0) return;
  const long long Tc = st->cost;
  const T gamma = (T)st->rs.gamma_cur;
  const int i0 = wg_first[w], i1 = wg_first[w + 1];
  if (i0 >= i1) return;
  VA rr[kBFMaxQ], pa[kBFMaxQ];
  int nv[kBFMaxQ];
  int kcur = -1, qcur = 0;
  long long moved = 0;
  auto flush = [&]() {
    const BInst& I = inst[kcur];
    const int nq = (I.m + VN - 1) / VN;
    const int lo = inst_lo[kcur], hi = inst_hi[kcur];
    const bool whole = bf_wg_of(item_pref[lo], Tc, G) == w && bf_wg_of(item_pref[hi], Tc, G) == w;
    T* dst = whole ? r_all + I.row_off : part + (size_t)(w + kcur) * pst;
#pragma unroll
    for (int q = 0; q < kBFMaxQ; ++q) {
      const int gi = q * kBFThreads + tid;
      if (q < qcur && gi < nq) {
        VA v = pa[q];
        if (whole) v += rr[q];
        *reinterpret_cast<VA*>(dst + (size_t)gi * VN) = v;
      }
    }
  };
  for (int i = i0; i < i1; ++i) {
    const BItem it = items[i];
    const BInst& I = inst[it.inst];
    const int nq = (I.m + VN - 1) / VN;
    const int qk = bf_q_of(nq);
    if (it.inst != kcur) {
      if (kcur >= 0) flush();
      kcur = it.inst;
      qcur = qk;
      const T* r = r_all + I.row_off;
#pragma unroll
      for (int q = 0; q < kBFMaxQ; ++q) {
        const int g = q * kBFThreads + tid;
        nv[q] = q < qk ? max(0, min(VN, I.m - g * VN)) : 0;
#pragma unroll
        for (int e = 0; e < VN; ++e) {
          rr[q][e] = (T)0;
          pa[q][e] = (T)0;
        }
        if (q < qk) {
          const VA v = *reinterpret_cast<const VA*>(r + (size_t)min(g, nq - 1) * VN);
#pragma unroll
          for (int e = 0; e < VN; ++e) rr[q][e] = e < nv[q] ? v[e] : (T)0;
        }
      }
    }
    BRParams bp = bp0;
    bp.lam = I.lam;
    bp.lam_eta = I.lam * bp0.eta;
    bp.c2 = 2.0 * I.c;
    bp.beta = I.beta;
    const int j00 = sel_cols[it.pos];
    const int C = bf_cols(qk);
    for (int cs = 0; cs < it.cnt; cs += C) {
      const int cnt = min(C, it.cnt - cs);
      switch (qk) {
        case 1:
          bf_group<T, 1>(I, nq, j00 + cs, cnt, rr, pa, nv, red, s_d, lane, wave, tid, gamma, bp,
                         x_all, cn2, moved);
          break;
        case 2:
          bf_group<T, 2>(I, nq, j00 + cs, cnt, rr, pa, nv, red, s_d, lane, wave, tid, gamma, bp,
                         x_all, cn2, moved);
          break;
        default:
          bf_group<T, 4>(I, nq, j00 + cs, cnt, rr, pa, nv, red, s_d, lane, wave, tid, gamma, bp,
                         x_all, cn2, moved);
          break;
      }
    }
  }
  if (kcur >= 0) flush();
  if (tid == 0 && moved)
    atomicAdd(reinterpret_cast<unsigned long long*>(&st->rs.moved_updates),
              (unsigned long long)moved);
}

// r_k += the partial slots (w + k), w = the workgroups that shared instance k's items, in
// workgroup order (instances held by one workgroup were written by it).  A workgroup whose
// share is empty (an item costing more than a share spans several thresholds) wrote no
// slot and is skipped.  One thread per row group; workgroup = one tile of 256 row groups of
// instance tile_inst[tile] (tile_base[k] = its first tile).  The slots' flags go to LDS first,
// so that every slot is then loaded unconditionally (a skipped one is read and discarded)
// and the loads of several slots are in flight together.
constexpr int kBRedSlots = 1024;  // slots flagged in LDS at a time
template <typename T>
__global__ void __launch_bounds__(256)
k_bfused_reduce(const BInst* __restrict__ inst, const int* __restrict__ tile_base,
                const int* __restrict__ tile_inst, const long long* __restrict__ item_pref,
                const int* __restrict__ wg_first, const int* __restrict__ inst_lo,
                const int* __restrict__ inst_hi, const BState* __restrict__ st, int G,
                int ntiles, const T* __restrict__ part, long long pst,
                T* __restrict__ r_all) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  __shared__ unsigned char s_on[kBRedSlots];
  if (st->items == 0) return;
  const long long Tc = st->cost;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int k = tile_inst[tile];
    const int ilo = inst_lo[k], ihi = inst_hi[k];
    if (ilo > ihi) continue;
    const int w0 = bf_wg_of(item_pref[ilo], Tc, G), w1 = bf_wg_of(item_pref[ihi], Tc, G);
    if (w0 == w1) continue;
    const BInst& I = inst[k];
    const int nq = (I.m + VN - 1) / VN;
    const int gi = min((tile - tile_base[k]) * 256 + (int)threadIdx.x, nq - 1);
    T* r = r_all + I.row_off + (size_t)gi * VN;
    VA s = *reinterpret_cast<const VA*>(r);
    for (int c0 = w0; c0 <= w1; c0 += kBRedSlots) {
      const int c1 = min(w1 + 1, c0 + kBRedSlots);
      __syncthreads();  // every thread is done with the previous flags
      for (int ww = c0 + (int)threadIdx.x; ww < c1; ww += 256)
        s_on[ww - c0] = wg_first[ww] < wg_first[ww + 1];
      __syncthreads();
      const T* pp = part + (size_t)(c0 + k) * pst + (size_t)gi * VN;
      int ww = c0;
      for (; ww + 4 <= c1; ww += 4, pp += 4 * pst) {
        VA v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const VA*>(pp + (size_t)u * pst);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (s_on[ww + u - c0]) s += v[u];
      }
      for (; ww < c1; ++ww, pp += pst)
        if (s_on[ww - c0]) s += *reinterpret_cast<const VA*>(pp);
    }
    if ((tile - tile_base[k]) * 256 + (int)threadIdx.x < nq) *reinterpret_cast<VA*>(r) = s;
  }
}

// ------------------------------------------------------------------ fold plan / tiles
// One workgroup: per instance, the range of the listed (ascending global) columns that
// belong to it, its column grouping and its tile count; tile offsets by a block scan.
template <int VN>
__global__ void __launch_bounds__(1024)
k_bfold_plan(int K, const BInst* __restrict__ inst, const int* __restrict__ J_idx,
             BState* __restrict__ st, int* __restrict__ J_lo, int* __restrict__ Jn,
             int* __restrict__ Gk, int* __restrict__ ngk, int* __restrict__ nrtk,
             int* __restrict__ tile_off) {
  __shared__ int sh[17];
  const int J = st->rs.J_cnt;
  int run = 0;
  for (int k0 = 0; k0 < K; k0 += 1024) {
    const int k = k0 + threadIdx.x;
    int tiles = 0;
    if (k < K) {
      const int c0 = inst[k].col_off, c1 = c0 + inst[k].n;
      int lo = 0, hi = J;  // first listed entry >= c0
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (J_idx[mid] < c0)
          lo = mid + 1;
        else
          hi = mid;
      }
      const int a = lo;
      hi = J;  // first listed entry >= c1
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (J_idx[mid] < c1)
          lo = mid + 1;
        else
          hi = mid;
      }
      const int cnt = lo - a;
      int G = (cnt + kBMaxGroups - 1) / kBMaxGroups;
      if (G < 16) G = 16;
      const int ng = (cnt + G - 1) / G;
      const int nrt = (inst[k].m + 256 * VN - 1) / (256 * VN);
      tiles = ng * nrt;
      J_lo[k] = a;
      Jn[k] = cnt;
      Gk[k] = G;
      ngk[k] = ng;
      nrtk[k] = nrt;
    }
    int tot;
    const int off = block_exclusive_scan_1024(tiles, sh, &tot);
    if (k < K) tile_off[k] = run + off;
    run += tot;
  }
  if (threadIdx.x == 0) {
    tile_off[K] = run;
    st->tiles = run;
  }
}

template <typename T, typename Acc>
__global__ void __launch_bounds__(256)
k_bfold_partial(int K, const BInst* __restrict__ inst, const int* __restrict__ J_idx,
                const T* __restrict__ J_val, const int* __restrict__ J_lo,
                const int* __restrict__ Jn, const int* __restrict__ Gk,
                const int* __restrict__ ngk, const int* __restrict__ nrtk,
                const int* __restrict__ tile_off, const BState* __restrict__ st,
                Acc* __restrict__ part, long long Mtot) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  const int ntiles = st->tiles;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int k = upper_idx(tile_off, K, tile);
    const BInst& I = inst[k];
    const int lt = tile - tile_off[k];
    const int nrt = nrtk[k];
    const int g = lt / nrt, rt = lt - g * nrt;
    const int G = Gk[k];
    const int e0 = J_lo[k] + g * G;
    const int e1 = min(e0 + G, J_lo[k] + Jn[k]);
    const T* A = (const T*)I.A;
    const int m = I.m;
    const int row0 = rt * 256 * VN + threadIdx.x * VN;
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
          const int j = J_idx[e + u] - I.col_off;
          d[u] = (Acc)J_val[e + u];
          a[u] = __builtin_nontemporal_load(
              reinterpret_cast<const VA*>(A + (size_t)j * I.lda + row0));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < VN; ++v) acc[v] += (Acc)a[u][v] * d[u];
      }
      for (; e < e1; ++e) {
        const int j = J_idx[e] - I.col_off;
        const Acc d = (Acc)J_val[e];
        const VA a = __builtin_nontemporal_load(
            reinterpret_cast<const VA*>(A + (size_t)j * I.lda + row0));
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[v] += (Acc)a[v] * d;
      }
    } else if (row0 < m) {
      for (int e = e0; e < e1; ++e) {
        const int j = J_idx[e] - I.col_off;
        const Acc d = (Acc)J_val[e];
        for (int v = 0; v < m - row0; ++v) acc[v] += (Acc)A[(size_t)j * I.lda + row0 + v] * d;
      }
    }
    if (row0 < m) {
      Acc* dst = part + (size_t)g * Mtot + I.row_off + row0;
      for (int v = 0; v < VN; ++v)
        if (row0 + v < m) dst[v] = acc[v];
    }
  }
}

template <typename TB, typename Acc, typename TO>
__global__ void __launch_bounds__(256)
k_bfold_reduce(const TB* __restrict__ base, double base_scale, const Acc* __restrict__ part,
               long long Mtot, const int* __restrict__ row_inst, const int* __restrict__ ngk,
               TO* __restrict__ out, double* __restrict__ out64) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < Mtot;
       i += (long long)gridDim.x * blockDim.x) {
    const int ng = ngk[row_inst[i]];
    Acc s = (Acc)(base_scale * (double)base[i]);
    for (int g = 0; g < ng; ++g) s += part[(size_t)g * Mtot + i];
    if (out) out[i] = (TO)s;
    if (out64) out64[i] = (double)s;
  }
}

// ------------------------------------------------------------------ checks
// One workgroup per instance: F_k (FP64 accumulation) from the residual rsrc, then the
// stopping test of the relative objective error.
//  mode 0: rsrc is a fresh FP64 residual; an active instance below the tolerance stops.
//  mode 1: rsrc is the running residual; an active instance below the tolerance becomes a
//          candidate (cand[k] = 1), to be confirmed with a fresh residual.
//  mode 2: rsrc is a fresh FP64 residual of the candidates; a candidate below the tolerance
//          stops, any other restarts its running residual rrun from the fresh one.
// A non-finite F stops the instance in every mode.
template <typename T, typename TR>
__global__ void __launch_bounds__(256)
k_bobj_check(int K, const BInst* __restrict__ inst, const TR* __restrict__ rsrc,
             const T* __restrict__ x_all, BRParams bp0, double tol, const BState* __restrict__ st,
             double* __restrict__ Fk, int* __restrict__ active, long long* __restrict__ done_round,
             int mode, int* __restrict__ cand, T* __restrict__ rrun) {
  __shared__ double res[3];
  __shared__ int s_restart;
  for (int k = blockIdx.x; k < K; k += gridDim.x) {
    if (mode == 2 && !cand[k]) continue;  // uniform over the workgroup
    const BInst& I = inst[k];
    BRParams bp = bp0;
    double sr = 0.0, sx = 0.0, sh = 0.0;
    for (int i = threadIdx.x; i < I.m; i += 256) {
      const double v = (double)rsrc[I.row_off + i];
      sr += v * v;
    }
    for (int j = threadIdx.x; j < I.n; j += 256) {
      const double v = (double)x_all[I.col_off + j];
      sx += v * v;
      sh += h_value<double>(v, bp);
    }
    block_sum3_256(sr, sx, sh, res);
    __syncthreads();
    if (threadIdx.x == 0) {
      const double F = 0.5 * res[0] - I.c * res[1] + I.lam * res[2];
      Fk[k] = F;
      s_restart = 0;
      const bool below = tol > 0.0 && I.F_star != 0.0 && (F - I.F_star) / fabs(I.F_star) <= tol;
      if (mode == 1) cand[k] = active[k] && below && isfinite(F);
      if (active[k]) {
        const bool stop = !isfinite(F) || (mode != 1 && below);
        if (stop) {
          active[k] = 0;
          done_round[k] = st->rs.k;
        } else if (mode == 2) {
          s_restart = 1;
        }
      }
      if (mode == 2) cand[k] = 0;
    }
    __syncthreads();
    if (s_restart)
      for (int i = threadIdx.x; i < I.m; i += 256) rrun[I.row_off + i] = (T)rsrc[I.row_off + i];
    __syncthreads();
  }
}

// v[j] = x[j] for the columns of candidate instances, 0 elsewhere (the fresh residual of the
// confirmation is then folded from the candidates' columns only).
template <typename T>
__global__ void k_bmask_cand(const T* __restrict__ x_all, const int* __restrict__ col_inst,
                             const int* __restrict__ cand, long long Ntot, T* __restrict__ v) {
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < Ntot;
       j += (long long)gridDim.x * blockDim.x)
    v[j] = cand[col_inst[j]] ? x_all[j] : (T)0;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_bprobe(const BInst* __restrict__ inst, const int* __restrict__ col_inst, long long Ntot,
         const double* __restrict__ r64, const T* __restrict__ x_all,
         const double* __restrict__ cn2, BRParams bp0, double* __restrict__ cm,
         double* __restrict__ cs, int* __restrict__ cz) {
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * 4;
  for (long long j = blockIdx.x * 4ll + (threadIdx.x >> 6); j < Ntot; j += nw) {
    const BInst& I = inst[col_inst[j]];
    const T* col = (const T*)I.A + (size_t)(j - I.col_off) * I.lda;
    const double dot = col_dot<T, double, double, 4>(col, r64 + I.row_off, I.m, lane);
    if (lane == 0) {
      BRParams bp = bp0;
      bp.lam = I.lam;
      bp.lam_eta = I.lam * bp0.eta;
      bp.c2 = 2.0 * I.c;
      bp.beta = I.beta;
      const double xj = (double)x_all[j];
      double g = dot - bp.c2 * xj;
      if (bp.reg) g -= bp.lam * dh_minus<double>(xj, bp);
      const double q = cn2[j] + I.tau;
      const double xh = soft_clip<double>(xj - g / q, bp.lam_eta / q, bp.beta);
      const double y = soft_clip<double>(xj - g, bp.lam_eta, bp.beta);
      cm[j] = fabs(xh - xj);
      cs[j] = (xj - y) * (xj - y);
      cz[j] = xh != 0.0;
    }
  }
}

__global__ void __launch_bounds__(256)
k_bprobe_reduce(int K, const BInst* __restrict__ inst, const double* __restrict__ cm,
                const double* __restrict__ cs, const int* __restrict__ cz,
                double* __restrict__ out /* 3 per instance */) {
  __shared__ double res[3];
  __shared__ double shm[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = blockIdx.x; k < K; k += gridDim.x) {
    const BInst& I = inst[k];
    double mx = 0.0, sm = 0.0, nz = 0.0;
    for (int j = threadIdx.x; j < I.n; j += 256) {
      mx = fmax(mx, cm[I.col_off + j]);
      sm += cs[I.col_off + j];
      nz += (double)cz[I.col_off + j];
    }
    const double wm = wave_max(mx);
    if (lane == 0) shm[wave] = wm;
    block_sum3_256(sm, nz, 0.0, res);
    __syncthreads();
    if (threadIdx.x == 0) {
      out[3 * k] = fmax(fmax(shm[0], shm[1]), fmax(shm[2], shm[3]));
      out[3 * k + 1] = sqrt(res[0]);
      out[3 * k + 2] = res[1];
    }
    __syncthreads();
  }
}

// Per-instance merit test after a probe: deactivate instances with merit <= tol.
__global__ void k_bmerit_check(int K, const double* __restrict__ pr, double tol,
                               const BState* __restrict__ st, int* __restrict__ active,
                               long long* __restrict__ done_round) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
    if (active[k] && pr[3 * k] <= tol) {
      active[k] = 0;
      done_round[k] = st->rs.k;
    }
  }
}

__global__ void k_binit(BState* st, long long k, double gamma, double mu, int Ntot, int K,
                        int* active, long long* done_round, long long* inst_upd, int reset) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < K; q += gridDim.x * blockDim.x) {
    if (reset) {
      active[q] = 1;
      done_round[q] = -1;
      inst_upd[q] = 0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rs.k = k;
    if (reset) {
      st->rs.coord_updates = 0;
      st->rs.moved_updates = 0;
    }
    st->rs.gamma_cur = gamma;
    st->rs.gamma_next = gamma;
    st->rs.gamma_mu = mu;
    st->rs.S_cnt = 0;
    st->rs.work_ctr = 0;
    st->rs.J_cnt = 0;
    st->rs.n_all = Ntot;
    st->items = 0;
    st->tiles = 0;
  }
}

template <typename T>
__global__ void k_bcolnorm2(const BInst* __restrict__ inst, const int* __restrict__ col_inst,
                            long long Ntot, double* __restrict__ cn2) {
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * 4;
  for (long long j = blockIdx.x * 4ll + (threadIdx.x >> 6); j < Ntot; j += nw) {
    const BInst& I = inst[col_inst[j]];
    const T* col = (const T*)I.A + (size_t)(j - I.col_off) * I.lda;
    double s = 0.0;
    for (int i = lane; i < I.m; i += 64) {
      const double v = (double)col[i];
      s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) cn2[j] = s;
  }
}

}  // namespace

namespace {

void batch_free(sca_batch* B) {
  void* ptrs[] = {B->d_inst, B->d_blk_inst, B->d_blk_col0, B->d_blk_len, B->d_blk_cols,
                  B->d_row_inst, B->d_col_inst, B->d_chunk_a, B->d_chunk_b, B->d_chunk_cnt,
                  B->d_cn2, B->d_b, B->d_r64, B->d_rrun, B->d_sel_cols, B->d_items,
                  B->d_dx_sel, B->d_J_idx, B->d_J_val, B->d_J_lo, B->d_Jn, B->d_G, B->d_ng, B->d_nrt,
                  B->d_tile_off, B->d_part, B->d_state, B->d_active, B->d_done, B->d_upd,
                  B->d_F, B->d_cm, B->d_cs, B->d_cz, B->d_pr, B->d_item_pref,
                  B->d_chunk_cost, B->d_wg_first, B->d_inst_lo, B->d_inst_hi,
                  B->d_tile_base, B->d_tile_inst, B->d_bpart, B->d_cand};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (B->graph) (void)hipGraphExecDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  adjoint_release(B->adj);
  B->adj = nullptr;
}

int* N_total_ptr(sca_batch* B) { return (int*)((char*)B->d_state + offsetof(RoundState, n_all)); }
int* S_ptr(sca_batch* B) { return (int*)((char*)B->d_state + offsetof(RoundState, S_cnt)); }

// Fold of the listed (J_idx, J_val) columns into out = base_scale*base + A_J d.
template <typename T, typename Acc, typename TB, typename TO>
void batch_fold(sca_batch* B, const TB* base, double base_scale, TO* out, double* out64,
                hipStream_t s) {
  constexpr int VN = V16<T>::N;
  hipLaunchKernelGGL(k_bfold_plan<VN>, dim3(1), dim3(1024), 0, s, B->K, (const BInst*)B->d_inst,
                     (const int*)B->d_J_idx, B->d_state, B->d_J_lo, B->d_Jn, B->d_G, B->d_ng,
                     B->d_nrt, B->d_tile_off);
  hipLaunchKernelGGL((k_bfold_partial<T, Acc>), dim3(8 * B->ncu), dim3(256), 0, s, B->K,
                     (const BInst*)B->d_inst, (const int*)B->d_J_idx, (const T*)B->d_J_val,
                     (const int*)B->d_J_lo, (const int*)B->d_Jn, (const int*)B->d_G,
                     (const int*)B->d_ng, (const int*)B->d_nrt, (const int*)B->d_tile_off,
                     (const BState*)B->d_state, (Acc*)B->d_part, B->Mtot);
  const int g = (int)std::min<long long>((B->Mtot + 255) / 256, 16ll * B->ncu);
  hipLaunchKernelGGL((k_bfold_reduce<TB, Acc, TO>), dim3(g), dim3(256), 0, s, base, base_scale,
                     (const Acc*)B->d_part, B->Mtot, (const int*)B->d_row_inst,
                     (const int*)B->d_ng, out, out64);
}

template <typename T>
void batch_compact(sca_batch* B, const T* v, const int* idx, const int* N_ptr, long long Nmax,
                   int count_moved, hipStream_t s) {
  const int nch = (int)((Nmax + kChunk - 1) / kChunk);
  const int cg = std::max(1, std::min(nch, 2 * B->ncu));
  hipLaunchKernelGGL(k_compact_count<T>, dim3(cg), dim3(1024), 0, s, v, N_ptr, B->d_chunk_cnt);
  hipLaunchKernelGGL(k_compact_scatter<T>, dim3(cg), dim3(1024), 0, s, v, idx, N_ptr,
                     (const int*)B->d_chunk_cnt, B->d_J_idx, (T*)B->d_J_val,
                     (RoundState*)B->d_state, count_moved);
}

int bf_grid(const sca_batch* B) { return B->bf_wg_per_cu * B->ncu; }

template <typename T>
void launch_bfused(sca_batch* B, T* x, T* r, const BRParams& bp, hipStream_t s) {
  hipLaunchKernelGGL((k_bfused<T>), dim3(bf_grid(B)), dim3(kBFThreads), 0, s,
                     (const BInst*)B->d_inst, (const BItem*)B->d_items,
                     (const long long*)B->d_item_pref, (const int*)B->d_wg_first,
                     (const int*)B->d_inst_lo, (const int*)B->d_inst_hi,
                     (const int*)B->d_sel_cols, r, x, (const double*)B->d_cn2, B->d_state,
                     (T*)B->d_bpart, B->bf_pst, bp);
}

template <typename T>
void batch_round(sca_batch* B, const sca_opts* o, T* x, T* r, hipStream_t s) {
  const uint64_t Tthr = selection_threshold(o->select_p);
  BRParams bp;
  bp.tau = 0;
  bp.lam = 0;
  bp.lam_eta = 0;
  bp.c2 = 0;
  bp.beta = INFINITY;
  bp.theta = B->theta;
  bp.eta = B->eta;
  bp.reg = B->reg;
  const bool fused = B->bf_kind == 1 && B->bf_q > 0;
  const int G = fused ? bf_grid(B) : 0;
  const int nch = (B->Btot + kChunk - 1) / kChunk;
  const int cg = std::max(1, std::min(nch, 2 * B->ncu));
  hipLaunchKernelGGL(k_bsel_count, dim3(cg), dim3(1024), 0, s, B->Btot, (const int*)B->d_blk_inst,
                     (const int*)B->d_blk_len, (const BInst*)B->d_inst, (const int*)B->d_active,
                     o->seed, Tthr, (const BState*)B->d_state, B->d_blk_cols, B->d_chunk_a,
                     B->d_chunk_b, B->d_chunk_cost, B->d_inst_lo, B->d_inst_hi, B->d_upd);
  hipLaunchKernelGGL(k_bsel_scatter, dim3(cg), dim3(1024), 0, s, B->Btot,
                     (const int*)B->d_blk_inst, (const int*)B->d_blk_col0,
                     (const int*)B->d_blk_cols, (const int*)B->d_chunk_a,
                     (const int*)B->d_chunk_b, (const long long*)B->d_chunk_cost,
                     (const BInst*)B->d_inst, B->d_state, B->d_sel_cols, B->d_items,
                     B->d_item_pref, B->d_wg_first, G, B->d_inst_lo, B->d_inst_hi);
  if (fused) {
    launch_bfused<T>(B, x, r, bp, s);
    const int g = std::max(1, std::min(B->bf_tiles, 16 * B->ncu));
    hipLaunchKernelGGL((k_bfused_reduce<T>), dim3(g), dim3(256), 0, s, (const BInst*)B->d_inst,
                       (const int*)B->d_tile_base, (const int*)B->d_tile_inst,
                       (const long long*)B->d_item_pref, (const int*)B->d_wg_first,
                       (const int*)B->d_inst_lo, (const int*)B->d_inst_hi,
                       (const BState*)B->d_state, G, B->bf_tiles, (const T*)B->d_bpart,
                       B->bf_pst, r);
    return;
  }
  hipLaunchKernelGGL((k_bgrad<T, 2>), dim3(2 * B->ncu), dim3(256), 0, s, (const BInst*)B->d_inst,
                     (const BItem*)B->d_items, (const int*)B->d_sel_cols, (const T*)r, x,
                     (const double*)B->d_cn2, B->d_state, (T*)B->d_dx_sel, bp);
  batch_compact<T>(B, (const T*)B->d_dx_sel, (const int*)B->d_sel_cols, (const int*)S_ptr(B),
                   B->Ntot, 1, s);
  batch_fold<T, T, T, T>(B, (const T*)r, 1.0, r, (double*)nullptr, s);
}

template <typename T>
void batch_residual(sca_batch* B, const T* x, T* r_out, hipStream_t s) {
  batch_compact<T>(B, x, (const int*)nullptr, (const int*)N_total_ptr(B), B->Ntot, 0, s);
  batch_fold<T, double, T, T>(B, (const T*)B->d_b, -1.0, r_out, B->d_r64, s);
}

BRParams batch_brparams(const sca_batch* B) {
  BRParams bp;
  bp.tau = 0;
  bp.lam = 0;
  bp.lam_eta = 0;
  bp.c2 = 0;
  bp.beta = INFINITY;
  bp.theta = B->theta;
  bp.eta = B->eta;
  bp.reg = B->reg;
  return bp;
}

template <typename T>
void batch_check(sca_batch* B, const T* x, double tol, hipStream_t s) {
  hipLaunchKernelGGL((k_bobj_check<T, double>), dim3(std::min(B->K, 4 * B->ncu)), dim3(256), 0,
                     s, B->K, (const BInst*)B->d_inst, (const double*)B->d_r64, x,
                     batch_brparams(B), tol, (const BState*)B->d_state, B->d_F, B->d_active,
                     B->d_done, 0, B->d_cand, (T*)nullptr);
}

// The relative-error test of sca_batch_solve from the running residual r; the instances
// below the tolerance are confirmed with a fresh FP64 residual folded from their own
// columns only (a failed confirmation restarts their running residual from it).
template <typename T>
void batch_check_running(sca_batch* B, const T* x, T* r, double tol, hipStream_t s) {
  const int gk = std::min(B->K, 4 * B->ncu);
  hipLaunchKernelGGL((k_bobj_check<T, T>), dim3(gk), dim3(256), 0, s, B->K,
                     (const BInst*)B->d_inst, (const T*)r, x, batch_brparams(B), tol,
                     (const BState*)B->d_state, B->d_F, B->d_active, B->d_done, 1, B->d_cand, r);
  const int g = (int)std::min<long long>((B->Ntot + 255) / 256, 16ll * B->ncu);
  hipLaunchKernelGGL(k_bmask_cand<T>, dim3(g), dim3(256), 0, s, x, (const int*)B->d_col_inst,
                     (const int*)B->d_cand, B->Ntot, (T*)B->d_dx_sel);
  batch_compact<T>(B, (const T*)B->d_dx_sel, (const int*)nullptr, (const int*)N_total_ptr(B),
                   B->Ntot, 0, s);
  batch_fold<T, double, T, T>(B, (const T*)B->d_b, -1.0, (T*)nullptr, B->d_r64, s);
  hipLaunchKernelGGL((k_bobj_check<T, double>), dim3(gk), dim3(256), 0, s, B->K,
                     (const BInst*)B->d_inst, (const double*)B->d_r64, x, batch_brparams(B), tol,
                     (const BState*)B->d_state, B->d_F, B->d_active, B->d_done, 2, B->d_cand, r);
}

template <typename T>
void batch_probe(sca_batch* B, const T* x, hipStream_t s) {
  hipLaunchKernelGGL(k_bprobe<T>, dim3(16 * B->ncu), dim3(256), 0, s, (const BInst*)B->d_inst,
                     (const int*)B->d_col_inst, B->Ntot, (const double*)B->d_r64, x,
                     (const double*)B->d_cn2, batch_brparams(B), B->d_cm, B->d_cs, B->d_cz);
  hipLaunchKernelGGL(k_bprobe_reduce, dim3(std::min(B->K, 4 * B->ncu)), dim3(256), 0, s, B->K,
                     (const BInst*)B->d_inst, (const double*)B->d_cm, (const double*)B->d_cs,
                     (const int*)B->d_cz, B->d_pr);
}

void batch_init(sca_batch* B, const sca_opts* o, int64_t k0, int reset, hipStream_t s) {
  const double g = gamma_at_round(o->gamma, o->gamma_mu, k0);
  hipLaunchKernelGGL(k_binit, dim3(std::max(1, (B->K + 255) / 256)), dim3(256), 0, s, B->d_state,
                     (long long)k0, g, o->gamma_mu, (int)B->Ntot, B->K, B->d_active, B->d_done,
                     B->d_upd, reset);
}

template <typename T>
void batch_rounds(sca_batch* B, const sca_opts* o, int64_t n, void* x, void* r, hipStream_t s) {
  for (int64_t i = 0; i < n; ++i) batch_round<T>(B, o, (T*)x, (T*)r, s);
}

sca_status check_hip(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(SCA_EHIP, "%s: %s", what, hipGetErrorString(e));
  return SCA_OK;
}

}  // namespace

void sca::batch_fresh_residual(sca_batch* B, const void* x, hipStream_t s) {
  if (B->dtype == SCA_F32)
    batch_residual<float>(B, (const float*)x, (float*)nullptr, s);
  else
    batch_residual<double>(B, (const double*)x, (double*)nullptr, s);
}

// ------------------------------------------------------------------ public entry points
extern "C" sca_status sca_batch_create(sca_batch** out, sca_dtype dtype, int64_t count,
                                       const sca_batch_item* items, void* stream) {
  if (!out) return set_error(SCA_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != SCA_F32 && dtype != SCA_F64) return set_error(SCA_EINVAL, "unknown dtype");
  if (count <= 0 || count > (1 << 20) || !items)
    return set_error(SCA_EINVAL, "count must lie in [1, 2^20] and items must not be NULL");
  const size_t es = dtype == SCA_F32 ? 4 : 8;
  const int64_t rpad = 16 / (int64_t)es;  // r offsets stay 16-byte aligned
  long long Mtot = 0, Ntot = 0, Btot = 0;
  for (int64_t k = 0; k < count; ++k) {
    const sca_batch_item& it = items[k];
    if (it.struct_size != sizeof(sca_batch_item))
      return set_error(SCA_EINVAL, "item %lld: struct_size mismatch", (long long)k);
    sca_status st = validate_problem_args(dtype, it.m, it.n, it.b_dev, it.lambda, it.c, it.beta,
                                          it.block_ptr_host, it.nblocks);
    if (st != SCA_OK) return set_error(st, "item %lld: %s", (long long)k, sca_last_error());
    if (!it.A_dev || ((uintptr_t)it.A_dev) % 16 || it.lda < it.m || (it.lda * (int64_t)es) % 16)
      return set_error(SCA_EINVAL, "item %lld: A must be 16-byte aligned, lda >= m, "
                       "lda*sizeof(element) a multiple of 16", (long long)k);
    if (!(it.tau >= 0.0) || !std::isfinite(it.tau))
      return set_error(SCA_EINVAL, "item %lld: tau must be finite and >= 0", (long long)k);
    if (!std::isfinite(it.F_star)) return set_error(SCA_EINVAL, "item %lld: F_star", (long long)k);
    Mtot += (it.m + rpad - 1) / rpad * rpad;
    Ntot += it.n;
    Btot += it.nblocks;
  }
  if (Mtot > INT32_MAX / 2 || Ntot > INT32_MAX / 2 || Btot > INT32_MAX / 2)
    return set_error(SCA_EINVAL, "batch too large (totals must stay below 2^30)");
  sca_batch* B = new (std::nothrow) sca_batch();
  if (!B) return set_error(SCA_ENOMEM, "host allocation failed");
  B->dtype = dtype;
  B->esize = es;
  B->K = (int)count;
  B->Mtot = Mtot;
  B->Ntot = Ntot;
  B->Btot = (int)Btot;
  B->ncu = device_cu_count();
  hipStream_t s = (hipStream_t)stream;
  std::vector<int> blk_inst, blk_col0, blk_len, row_inst(Mtot), col_inst(Ntot);
  blk_inst.reserve(Btot);
  blk_col0.reserve(Btot);
  blk_len.reserve(Btot);
  long long ro = 0, co = 0;
  int bo = 0;
  B->xoff.push_back(0);
  B->roff.push_back(0);
  for (int64_t k = 0; k < count; ++k) {
    const sca_batch_item& it = items[k];
    BInst I;
    I.A = it.A_dev;
    I.lda = it.lda;
    I.m = (int)it.m;
    I.n = (int)it.n;
    I.row_off = (int)ro;
    I.col_off = (int)co;
    I.blk_off = bo;
    I.nblk = (int)it.nblocks;
    I.lam = it.lambda;
    I.c = it.c;
    I.beta = it.beta;
    I.tau = it.tau;
    I.F_star = it.F_star;
    I.inst_id = it.instance;
    I.pad = 0;
    B->hinst.push_back(I);
    for (int64_t i = 0; i < it.nblocks; ++i) {
      blk_inst.push_back((int)k);
      blk_col0.push_back((int)(co + it.block_ptr_host[i]));
      blk_len.push_back((int)(it.block_ptr_host[i + 1] - it.block_ptr_host[i]));
    }
    const int64_t mp = (it.m + rpad - 1) / rpad * rpad;
    for (int64_t i = 0; i < mp; ++i) row_inst[ro + i] = (int)k;
    for (int64_t j = 0; j < it.n; ++j) col_inst[co + j] = (int)k;
    ro += mp;
    co += it.n;
    bo += (int)it.nblocks;
    B->xoff.push_back(co);
    B->roff.push_back(ro);
  }
  sca_status st = SCA_OK;
  const int nchB = (int)((Btot + kChunk - 1) / kChunk) + 1;
  const int nchN = (int)((Ntot + kChunk - 1) / kChunk) + 1;
#define BALLOC(ptr, bytes)                                              \
  if (st == SCA_OK) st = dev_alloc((void**)&(ptr), (bytes));
  BALLOC(B->d_inst, sizeof(BInst) * count);
  BALLOC(B->d_blk_inst, sizeof(int) * Btot);
  BALLOC(B->d_blk_col0, sizeof(int) * Btot);
  BALLOC(B->d_blk_len, sizeof(int) * Btot);
  BALLOC(B->d_blk_cols, sizeof(int) * Btot);
  BALLOC(B->d_row_inst, sizeof(int) * Mtot);
  BALLOC(B->d_col_inst, sizeof(int) * Ntot);
  BALLOC(B->d_chunk_a, sizeof(int) * nchB);
  BALLOC(B->d_chunk_b, sizeof(int) * nchB);
  BALLOC(B->d_chunk_cnt, sizeof(int) * nchN);
  BALLOC(B->d_cn2, sizeof(double) * Ntot);
  BALLOC(B->d_b, es * Mtot);
  BALLOC(B->d_r64, sizeof(double) * Mtot);
  BALLOC(B->d_rrun, es * Mtot + 16);
  BALLOC(B->d_sel_cols, sizeof(int) * Ntot);
  BALLOC(B->d_items, sizeof(BItem) * Ntot);
  BALLOC(B->d_dx_sel, es * Ntot);
  BALLOC(B->d_J_idx, sizeof(int) * Ntot);
  BALLOC(B->d_J_val, es * Ntot);
  BALLOC(B->d_J_lo, sizeof(int) * count);
  BALLOC(B->d_Jn, sizeof(int) * count);
  BALLOC(B->d_G, sizeof(int) * count);
  BALLOC(B->d_ng, sizeof(int) * count);
  BALLOC(B->d_nrt, sizeof(int) * count);
  BALLOC(B->d_tile_off, sizeof(int) * (count + 1));
  BALLOC(B->d_part, sizeof(double) * kBMaxGroups * Mtot);
  BALLOC(B->d_state, sizeof(BState));
  BALLOC(B->d_active, sizeof(int) * count);
  BALLOC(B->d_done, sizeof(long long) * count);
  BALLOC(B->d_upd, sizeof(long long) * count);
  BALLOC(B->d_F, sizeof(double) * count);
  BALLOC(B->d_cm, sizeof(double) * Ntot);
  BALLOC(B->d_cs, sizeof(double) * Ntot);
  BALLOC(B->d_cz, sizeof(int) * Ntot);
  BALLOC(B->d_pr, sizeof(double) * 3 * count);
  // fused round: where every instance's column fits the registers of a 256-thread workgroup
  {
    const long long VN = 16 / (long long)es;
    long long mmax = 0;
    for (int64_t k = 0; k < count; ++k) mmax = std::max<long long>(mmax, items[k].m);
    const long long nq = (mmax + VN - 1) / VN;
    const long long q = (nq + kBFThreads - 1) / kBFThreads;
    B->bf_q = q <= 1 ? 1 : q <= 2 ? 2 : q <= kBFMaxQ ? 4 : 0;
    B->bf_pst = (mmax + VN - 1) / VN * VN;
    B->bf_gmax = kBFMaxWgPerCu * B->ncu;
  }
  BALLOC(B->d_item_pref, sizeof(long long) * (Ntot + 1));
  BALLOC(B->d_chunk_cost, sizeof(long long) * nchB);
  BALLOC(B->d_wg_first, sizeof(int) * (B->bf_gmax + 1));
  BALLOC(B->d_inst_lo, sizeof(int) * count);
  BALLOC(B->d_inst_hi, sizeof(int) * count);
  BALLOC(B->d_tile_base, sizeof(int) * (count + 1));
  std::vector<int> tb(count + 1, 0);  // first fused-reduction tile (256 row groups) per instance
  for (int64_t k = 0; k < count; ++k) {
    const long long nq = (items[k].m + 16 / (long long)es - 1) / (16 / (long long)es);
    tb[k + 1] = tb[k] + (int)((nq + 255) / 256);
  }
  BALLOC(B->d_tile_inst, sizeof(int) * std::max(1, tb[count]));
  BALLOC(B->d_cand, sizeof(int) * count);
  if (B->bf_q > 0)
    BALLOC(B->d_bpart, es * (size_t)B->bf_pst * (B->bf_gmax + count));
#undef BALLOC
  if (st == SCA_OK) {
    bool ok = hipMemcpy(B->d_inst, B->hinst.data(), sizeof(BInst) * count,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_blk_inst, blk_inst.data(), sizeof(int) * Btot,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_blk_col0, blk_col0.data(), sizeof(int) * Btot,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_blk_len, blk_len.data(), sizeof(int) * Btot,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_row_inst, row_inst.data(), sizeof(int) * Mtot,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_col_inst, col_inst.data(), sizeof(int) * Ntot,
                        hipMemcpyHostToDevice) == hipSuccess;
    B->bf_tiles = tb[count];
    std::vector<int> ti(std::max(1, tb[count]), 0);
    for (int64_t k = 0; k < count; ++k)
      for (int t = tb[k]; t < tb[k + 1]; ++t) ti[t] = (int)k;
    ok = ok && hipMemcpy(B->d_tile_base, tb.data(), sizeof(int) * (count + 1),
                         hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(B->d_tile_inst, ti.data(), sizeof(int) * ti.size(),
                   hipMemcpyHostToDevice) == hipSuccess;
    // padding rows of b, r and the fold partials stay zero
    ok = ok && hipMemsetAsync(B->d_b, 0, es * Mtot, s) == hipSuccess &&
         hipMemsetAsync(B->d_rrun, 0, es * Mtot + 16, s) == hipSuccess &&
         hipMemsetAsync(B->d_part, 0, sizeof(double) * kBMaxGroups * Mtot, s) == hipSuccess &&
         hipMemsetAsync(B->d_r64, 0, sizeof(double) * Mtot, s) == hipSuccess &&
         hipMemsetAsync(B->d_cand, 0, sizeof(int) * count, s) == hipSuccess;
    for (int64_t k = 0; ok && k < count; ++k)
      ok = hipMemcpyAsync((char*)B->d_b + es * B->roff[k], items[k].b_dev, es * items[k].m,
                          hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (!ok) st = set_error(SCA_EHIP, "batch set-up copies failed");
  }
  if (st == SCA_OK) {
    hipLaunchKernelGGL(k_binit, dim3(std::max(1, (B->K + 255) / 256)), dim3(256), 0, s,
                       B->d_state, 0ll, 1.0, 0.0, (int)B->Ntot, B->K, B->d_active, B->d_done,
                       B->d_upd, 1);
    if (dtype == SCA_F32)
      hipLaunchKernelGGL(k_bcolnorm2<float>, dim3(16 * B->ncu), dim3(256), 0, s,
                         (const BInst*)B->d_inst, (const int*)B->d_col_inst, B->Ntot, B->d_cn2);
    else
      hipLaunchKernelGGL(k_bcolnorm2<double>, dim3(16 * B->ncu), dim3(256), 0, s,
                         (const BInst*)B->d_inst, (const int*)B->d_col_inst, B->Ntot, B->d_cn2);
    std::vector<double> cn2(Ntot);
    if (hipMemcpyAsync(cn2.data(), B->d_cn2, sizeof(double) * Ntot, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = set_error(SCA_EHIP, "batch column norms failed");
    for (int64_t k = 0; st == SCA_OK && k < count; ++k) {
      for (long long j = B->xoff[k]; j < B->xoff[k + 1]; ++j) {
        if (!std::isfinite(cn2[j])) {
          st = set_error(SCA_EINVAL, "item %lld: A holds NaN or Inf", (long long)k);
          break;
        }
        if (!(cn2[j] + B->hinst[k].tau > 0.0)) {
          st = set_error(SCA_EINVAL, "item %lld: a zero column with tau = 0", (long long)k);
          break;
        }
      }
    }
  }
  if (st == SCA_OK) {  // launch shape: the tuning table's batch row, else the default
    sca_launch l;
    long long mmax = 0;
    for (int64_t k = 0; k < count; ++k) mmax = std::max<long long>(mmax, items[k].m);
    if (batch_tuning(dtype, mmax, &l) && (l.grad_kind == 0 || B->bf_q > 0)) {
      B->bf_kind = l.grad_kind;
      if (l.grad_kind == 1) {
        B->bf_wg_per_cu = l.grad_wg_per_cu;
      }
    }
  }
  if (st == SCA_OK && hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess)
    st = set_error(SCA_EHIP, "stream creation failed");
  if (st != SCA_OK) {
    batch_free(B);
    delete B;
    return st;
  }
  *out = B;
  return SCA_OK;
}

extern "C" void sca_batch_destroy(sca_batch* B) {
  if (!B) return;
  batch_free(B);
  delete B;
}

extern "C" sca_status sca_batch_get_launch(sca_batch* B, sca_launch* out) {
  if (!B || !out) return set_error(SCA_EINVAL, "NULL argument");
  out->struct_size = sizeof(sca_launch);
  out->grad_kind = (B->bf_kind == 1 && B->bf_q > 0) ? 1 : 0;
  out->grad_cols = kBFSlots;
  out->grad_unroll = 1;
  out->grad_wg_per_cu = B->bf_wg_per_cu;
  return SCA_OK;
}

extern "C" sca_status sca_batch_set_launch(sca_batch* B, const sca_launch* l) {
  if (!B || !l) return set_error(SCA_EINVAL, "NULL argument");
  if (l->struct_size != sizeof(sca_launch)) return set_error(SCA_EINVAL, "struct_size mismatch");
  if (l->grad_kind != 0 && l->grad_kind != 1)
    return set_error(SCA_EINVAL, "batch grad_kind must be 0 (two-pass) or 1 (fused)");
  if (l->grad_kind == 1) {
    if (B->bf_q == 0)
      return set_error(SCA_EINVAL, "the fused round needs every m <= %d (this dtype)",
                       kBFThreads * kBFMaxQ * (int)(16 / B->esize));
    if (l->grad_cols != kBFSlots)
      return set_error(SCA_EINVAL, "fused batch round: grad_cols must be %d (the kernel groups "
                       "8, 4 or 1 columns by the instance's m)", kBFSlots);
    if (l->grad_wg_per_cu < 1 || l->grad_wg_per_cu > kBFMaxWgPerCu)
      return set_error(SCA_EINVAL, "fused batch round: grad_wg_per_cu must lie in [1, %d]",
                       kBFMaxWgPerCu);
    B->bf_wg_per_cu = l->grad_wg_per_cu;
  }
  B->bf_kind = l->grad_kind;
  if (B->graph) {  // the cached solve graph holds the old launch shape
    (void)hipGraphExecDestroy(B->graph);
    B->graph = nullptr;
  }
  return SCA_OK;
}

extern "C" sca_status sca_batch_layout(sca_batch* B, int64_t* x_off, int64_t* r_off) {
  if (!B) return set_error(SCA_EINVAL, "batch is NULL");
  for (int k = 0; k <= B->K; ++k) {
    if (x_off) x_off[k] = B->xoff[k];
    if (r_off) r_off[k] = B->roff[k];
  }
  return SCA_OK;
}

extern "C" sca_status sca_batch_set_regularizer(sca_batch* B, sca_reg reg, double theta) {
  if (!B) return set_error(SCA_EINVAL, "batch is NULL");
  if (reg == SCA_REG_L1) {
    B->reg = 0;
    B->theta = 0;
    B->eta = 1;
  } else if (reg == SCA_REG_EXP || reg == SCA_REG_LOG) {
    if (!(theta > 0.0) || !std::isfinite(theta)) return set_error(SCA_EINVAL, "theta must be > 0");
    B->reg = (int)reg;
    B->theta = theta;
    B->eta = reg == SCA_REG_EXP ? theta : theta / std::log1p(theta);
  } else {
    return set_error(SCA_EINVAL, "unknown regulariser");
  }
  if (B->graph) {
    (void)hipGraphExecDestroy(B->graph);
    B->graph = nullptr;
  }
  return SCA_OK;
}

extern "C" sca_status sca_batch_residual(sca_batch* B, const void* x, void* r, void* stream) {
  if (!B || !x || !r) return set_error(SCA_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if (B->dtype == SCA_F32)
    batch_residual<float>(B, (const float*)x, (float*)r, s);
  else
    batch_residual<double>(B, (const double*)x, (double*)r, s);
  return check_hip("sca_batch_residual");
}

extern "C" sca_status sca_batch_step(sca_batch* B, const sca_opts* o, int64_t round_begin,
                                     int64_t nrounds, void* x, void* r, void* stream) {
  if (!B) return set_error(SCA_EINVAL, "batch is NULL");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if (o->delay_chunks > 1 || o->async_workgroups > 0)
    return set_error(SCA_EINVAL,
                     "bounded-delay and lock-free rounds need the single-problem dense path");
  if (round_begin < 0 || nrounds < 0 || !x || !r)
    return set_error(SCA_EINVAL, "bad round range or NULL x / r");
  if (((uintptr_t)r) % 16 || ((uintptr_t)x) % B->esize)
    return set_error(SCA_EINVAL, "x or r misaligned");
  hipStream_t s = (hipStream_t)stream;
  batch_init(B, o, round_begin, 1, s);
  if (B->dtype == SCA_F32)
    batch_rounds<float>(B, o, nrounds, x, r, s);
  else
    batch_rounds<double>(B, o, nrounds, x, r, s);
  return check_hip("sca_batch_step");
}

extern "C" sca_status sca_batch_objective(sca_batch* B, const sca_opts* o, const void* x,
                                          double* F, double* merit, double* MF, int64_t* nnz,
                                          void* stream) {
  if (!B || !x) return set_error(SCA_EINVAL, "NULL argument");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (B->dtype == SCA_F32) {
    batch_residual<float>(B, (const float*)x, (float*)nullptr, s);
    batch_check<float>(B, (const float*)x, 0.0, s);
    batch_probe<float>(B, (const float*)x, s);
  } else {
    batch_residual<double>(B, (const double*)x, (double*)nullptr, s);
    batch_check<double>(B, (const double*)x, 0.0, s);
    batch_probe<double>(B, (const double*)x, s);
  }
  std::vector<double> hF(B->K), hp(3 * B->K);
  if (hipMemcpyAsync(hF.data(), B->d_F, sizeof(double) * B->K, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(hp.data(), B->d_pr, sizeof(double) * 3 * B->K, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "batch objective: %s", hipGetErrorString(hipGetLastError()));
  for (int k = 0; k < B->K; ++k) {
    if (F) F[k] = hF[k];
    if (merit) merit[k] = hp[3 * k];
    if (MF) MF[k] = hp[3 * k + 1];
    if (nnz) nnz[k] = (int64_t)hp[3 * k + 2];
  }
  return SCA_OK;
}

// E rounds followed by the per-instance stopping tests: the relative objective error from
// the running residual, confirmed with a fresh one (as sca_solve does); with tol_merit > 0
// a fresh FP64 residual of every instance for both tests and the merit.
template <typename T>
static void batch_cycle(sca_batch* B, const sca_opts* o, T* x, T* r, hipStream_t s) {
  for (int64_t i = 0; i < o->check_every; ++i) batch_round<T>(B, o, x, r, s);
  if (o->tol_merit <= 0.0) {
    batch_check_running<T>(B, x, r, o->tol_rel_obj, s);
    return;
  }
  batch_residual<T>(B, x, (T*)nullptr, s);
  batch_check<T>(B, x, o->tol_rel_obj, s);
  {
    batch_probe<T>(B, x, s);
    hipLaunchKernelGGL(k_bmerit_check, dim3(std::max(1, (B->K + 255) / 256)), dim3(256), 0, s,
                       B->K, (const double*)B->d_pr, o->tol_merit, (const BState*)B->d_state,
                       B->d_active, B->d_done);
  }
}

extern "C" sca_status sca_batch_solve(sca_batch* B, const sca_opts* o, void* x,
                                      sca_stats* stats, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!B || !x) return set_error(SCA_EINVAL, "NULL argument");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if (o->delay_chunks > 1 || o->async_workgroups > 0)
    return set_error(SCA_EINVAL,
                     "bounded-delay and lock-free rounds need the single-problem dense path");
  if (o->max_rounds < 0 || o->check_every < 1)
    return set_error(SCA_EINVAL, "max_rounds >= 0 and check_every >= 1");
  if (stats)
    for (int k = 0; k < B->K; ++k)
      if (stats[k].struct_size != sizeof(sca_stats))
        return set_error(SCA_EINVAL, "stats[%d].struct_size mismatch", k);
  if (o->tol_rel_obj > 0.0)
    for (int k = 0; k < B->K; ++k)
      if (B->hinst[k].F_star == 0.0)
        return set_error(SCA_EINVAL, "instance %d: tol_rel_obj needs a nonzero F_star", k);
  hipStream_t s = (hipStream_t)stream;
  void* r = B->d_rrun;
  batch_init(B, o, 0, 1, s);
  if (B->dtype == SCA_F32)
    batch_residual<float>(B, (const float*)x, (float*)r, s);
  else
    batch_residual<double>(B, (const double*)x, (double*)r, s);
  // one graph = check_every rounds + check; built once per (x, check_every, tol)
  if (!B->graph || B->graph_rounds != o->check_every || B->graph_x != x ||
      B->graph_tol != o->tol_rel_obj || B->graph_tol_merit != o->tol_merit ||
      B->graph_p != o->select_p || B->graph_seed != o->seed) {
    if (B->graph) {
      (void)hipGraphExecDestroy(B->graph);
      B->graph = nullptr;
    }
    hipGraph_t g;
    if (hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(SCA_EHIP, "graph capture failed to start");
    if (B->dtype == SCA_F32)
      batch_cycle<float>(B, o, (float*)x, (float*)r, B->cap);
    else
      batch_cycle<double>(B, o, (double*)x, (double*)r, B->cap);
    if (hipStreamEndCapture(B->cap, &g) != hipSuccess)
      return set_error(SCA_EHIP, "graph capture failed");
    const hipError_t e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      B->graph = nullptr;
      return set_error(SCA_EHIP, "graph instantiation failed");
    }
    B->graph_rounds = (int)o->check_every;
    B->graph_x = x;
    B->graph_tol = o->tol_rel_obj;
    B->graph_tol_merit = o->tol_merit;
    B->graph_p = o->select_p;
    B->graph_seed = o->seed;
  }
  std::vector<int> act(B->K);
  int64_t k = 0;
  int checks = 0;
  int nact = B->K;
  while (k < o->max_rounds && nact > 0) {
    if (hipGraphLaunch(B->graph, s) != hipSuccess)
      return set_error(SCA_EHIP, "graph launch failed");
    k += o->check_every;
    ++checks;
    if (hipMemcpyAsync(act.data(), B->d_active, sizeof(int) * B->K, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return set_error(SCA_EHIP, "batch solve: %s", hipGetErrorString(hipGetLastError()));
    nact = 0;
    for (int q = 0; q < B->K; ++q) nact += act[q];
  }
  // final report
  std::vector<double> F(B->K), mer(B->K), mf(B->K);
  std::vector<int64_t> nnz(B->K);
  if ((st = sca_batch_objective(B, o, x, F.data(), mer.data(), mf.data(), nnz.data(), stream)) !=
      SCA_OK)
    return st;
  std::vector<long long> done(B->K), upd(B->K);
  long long moved_all = 0;
  if (hipMemcpy(done.data(), B->d_done, sizeof(long long) * B->K, hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(upd.data(), B->d_upd, sizeof(long long) * B->K, hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(&moved_all, (char*)B->d_state + offsetof(RoundState, moved_updates),
                sizeof(long long), hipMemcpyDeviceToHost) != hipSuccess)
    return set_error(SCA_EHIP, "batch stats copy failed");
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int notconv = 0;
  for (int q = 0; q < B->K; ++q) {
    const bool conv = done[q] >= 0;
    const bool fin = std::isfinite(F[q]);
    const bool want = o->tol_rel_obj > 0.0 || o->tol_merit > 0.0;
    if (!conv && want) ++notconv;
    if (stats) {
      sca_stats& S = stats[q];
      S.rounds = conv ? done[q] : k;
      S.coord_updates = upd[q];
      S.moved_updates = moved_all;
      S.F = F[q];
      S.merit = mer[q];
      S.MF = mf[q];
      const double fs = B->hinst[q].F_star;
      S.rel_err = fs != 0.0 ? (F[q] - fs) / std::fabs(fs) : 0.0;
      S.seconds = secs;
      S.nnz = nnz[q];
      S.status = !fin ? SCA_ENONFINITE : ((!conv && want) ? SCA_ENOTCONV : SCA_OK);
      S.checks = checks;
    }
  }
  if (notconv) return set_error(SCA_ENOTCONV, "%d instances did not reach the tolerance", notconv);
  return SCA_OK;
}

extern "C" sca_status sca_batch_update_rhs(sca_batch* B, const void* b_all, const double* lambda,
                                           void* stream) {
  if (!B || !b_all || !lambda) return set_error(SCA_EINVAL, "NULL argument");
  for (int k = 0; k < B->K; ++k)
    if (!(lambda[k] >= 0.0) || !std::isfinite(lambda[k]))
      return set_error(SCA_EINVAL, "lambda[%d] must be finite and >= 0", k);
  hipStream_t s = (hipStream_t)stream;
  for (int k = 0; k < B->K; ++k) {  // copy the valid rows only; padding stays zero
    const size_t off = B->esize * (size_t)B->roff[k];
    if (hipMemcpyAsync((char*)B->d_b + off, (const char*)b_all + off,
                       B->esize * (size_t)B->hinst[k].m, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return set_error(SCA_EHIP, "rhs copy failed");
    B->hinst[k].lam = lambda[k];
  }
  if (hipMemcpyAsync(B->d_inst, B->hinst.data(), sizeof(BInst) * B->K, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "descriptor update failed");
  return SCA_OK;
}

extern "C" sca_status sca_batch_set_fstar(sca_batch* B, const double* F_star) {
  if (!B || !F_star) return set_error(SCA_EINVAL, "NULL argument");
  for (int k = 0; k < B->K; ++k) {
    if (!std::isfinite(F_star[k])) return set_error(SCA_EINVAL, "F_star[%d] not finite", k);
    B->hinst[k].F_star = F_star[k];
  }
  if (hipMemcpy(B->d_inst, B->hinst.data(), sizeof(BInst) * B->K, hipMemcpyHostToDevice) !=
      hipSuccess)
    return set_error(SCA_EHIP, "descriptor update failed");
  return SCA_OK;
}
