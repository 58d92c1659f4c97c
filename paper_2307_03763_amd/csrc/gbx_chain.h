// Independent-proposal chain kernel (device code); included by the host-side translation
// unit only, since it is not a template.
#pragma once
#include "gbx_kernels.h"

namespace gbx {

// Independent-proposal Metropolis-Hastings chain of one window per workgroup (Algorithm 4),
// in logarithmic depth.  With pi_i = logL_i - log_g_i and key_i = pi_i - T ln u_i, the chain
// moves from its current state c to the first later proposal j with key_j > pi_c (then
// u_j < exp((pi_j - pi_c) / T)); so with next(i) = min{ j > i : key_j > pi_i } the visited
// states are 0, next(0), next(next(0)), ... and the state after step i is the last of them
// not beyond i.  The kernel finds next(i) for every i with a max-tree over the keys, builds
// binary-lifting tables next^(2^k), and resolves every step from them; the decisions are the
// same comparisons (pi_c < key_j, in FP64, no contraction) as a step-by-step chain.
struct ChainWin {
  int64_t tree_off;  // doubles: max-tree, leaves at [P, 2P)
  int64_t jump_off;  // int32: K levels of n + 1 entries
  int64_t P;         // power of two >= n
  int32_t K, pad;    // 2^K > n
};

__global__ void __launch_bounds__(1024) k_mh_chain(const DevWin* __restrict__ wins, const ChainWin* __restrict__ cws,
                                                   const double* __restrict__ logL, const double* __restrict__ log_g,
                                                   const double* __restrict__ u, double temp, double* tree_all,
                                                   int32_t* jump_all, int32_t* __restrict__ chain,
                                                   int64_t* __restrict__ n_accept) {
  __shared__ unsigned s_acc;
  const DevWin w = wins[blockIdx.x];
  const ChainWin cw = cws[blockIdx.x];
  const int64_t n = w.n_cand, base = w.cand_off;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (n <= 0) {
    if (tid == 0) n_accept[blockIdx.x] = 0;
    return;
  }
  double* tree = tree_all + cw.tree_off;
  int32_t* jump = jump_all + cw.jump_off;
  const int64_t P = cw.P, n1 = n + 1;
  if (tid == 0) s_acc = 0u;
  // leaves; index 0 (the initial state) and padding can never be moved to, nor can a NaN key
  for (int64_t i = tid; i < P; i += nt) {
    double key = -__builtin_inf();
    if (i >= 1 && i < n) {
      const double pii = logL[base + i] - log_g[base + i];
      const double k = __dsub_rn(pii, __dmul_rn(temp, log(u[base + i])));
      if (k == k) key = k;
    }
    tree[P + i] = key;
  }
  __syncthreads();
  for (int64_t lvl = P >> 1; lvl >= 1; lvl >>= 1) {
    for (int64_t v = lvl + tid; v < 2 * lvl; v += nt) {
      const double a = tree[2 * v], b = tree[2 * v + 1];
      tree[v] = a > b ? a : b;
    }
    __syncthreads();
  }
  // next(i): the nearest right sibling subtree whose maximum exceeds pi_i, then its leftmost
  // leaf above pi_i (a NaN pi_i exceeds nothing: no move)
  for (int64_t i = tid; i < n; i += nt) {
    const double x = logL[base + i] - log_g[base + i];
    int64_t r = n;
    if (i + 1 < n && tree[P + i + 1] > x) {
      r = i + 1;
    } else {
      int64_t v = P + i;
      bool found = false;
      while (v > 1) {
        if (!(v & 1) && tree[v + 1] > x) {
          v = v + 1;
          found = true;
          break;
        }
        v >>= 1;
      }
      if (found) {
        while (v < P) {
          v <<= 1;
          if (!(tree[v] > x)) v += 1;
        }
        r = v - P;
      }
    }
    jump[i] = (int32_t)r;
  }
  if (tid == 0) jump[n] = (int32_t)n;
  __syncthreads();
  for (int k = 1; k < cw.K; ++k) {
    const int32_t* jp = jump + (int64_t)(k - 1) * n1;
    int32_t* jk = jump + (int64_t)k * n1;
    for (int64_t v = tid; v < n1; v += nt) jk[v] = jp[jp[v]];
    __syncthreads();
  }
  // state after step i: the furthest visited state not beyond i
  unsigned acc = 0;
  for (int64_t i = tid; i < n; i += nt) {
    int64_t x = 0;
    for (int k = cw.K - 1; k >= 0; --k) {
      const int64_t y = jump[(int64_t)k * n1 + x];
      if (y <= i) x = y;
    }
    chain[base + i] = (int32_t)x;
    acc += (x == i && i > 0) ? 1u : 0u;
  }
  if (acc) atomicAdd(&s_acc, acc);
  __syncthreads();
  if (tid == 0) n_accept[blockIdx.x] = (int64_t)s_acc;
}

}  // namespace gbx
