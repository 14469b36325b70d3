// Negacyclic number-theoretic transforms for gfx950.
//
// NTT over an RNS prime p (2^53 < p < 2^54): one workgroup per row of N
// residues, each thread holding E = 2^EL residues in registers.  The log2(N)
// butterfly stages run in register passes of EL stages (the last pass takes
// the rest); between passes the row goes through LDS (padded by one word every
// 32 so that the strided pass patterns spread over banks).  A last pass of a
// single stage reads or writes global memory straight from registers.
// Forward: Cooley-Tukey with the bit-reversed power table psi^brv(k), output
// in bit-reversed evaluation order.  Inverse: Gentleman-Sande with psi^-brv(k)
// and a final N^-1.  One Shoup product per butterfly, with a quotient that may
// be 2 short, so its result lies in [0, 4p) for any 64-bit input.  Forward
// butterflies are not reduced at all: (U, V) -> (U + V, U - V + 4p) with
// V < 4p raises the bound by 4p per stage, so reduced inputs stay below
// (1 + 4 log2 N) p <= 57p < 2^60 and the output is reduced once at the store.
// Inverse sums are not reduced inside a pass; each pass but the last brings
// its words back below 4p at its end, the last leaves them below 2^EL 4p for
// the final N^-1 product.
//
// Transforms over t = 65537 (batch encoding of slots and of the server bit
// planes) use the same register passes with 32-bit residues; decoding, which
// is not on the server path, is a radix-2 loop over LDS.
#include "kernels.hpp"

namespace pepsi {
namespace {

// Each thread holds E = 2^EL residues of a row; a row's log N stages run as passes of EL stages
// (the last pass takes what is left), with one exchange through padded LDS between passes.
// A row fills 64 KiB of LDS at N = 8192, so a CU holds two rows at a time: with 8 residues per
// thread (1024 threads, 16 waves per row) that is 8 waves per SIMD to hide latency, against 4
// with 16 residues, for one more exchange. Eight waves per SIMD need at most 64 VGPRs, which the
// inverse transforms are held to (ntt_waves). The transforms over t keep 16 residues.
template <int LOGN>
constexpr int ntt_el() { return LOGN == 13 ? 3 : 4; }
template <int EL>
constexpr int ntt_waves() { return EL == 3 ? 8 : 1; }   // minimum waves per SIMD (1: no bound)
template <int LOGN>
constexpr int ntt_t_el() { return 4; }
// Whether a last pass of d stages reads or writes global memory from registers (each thread then
// moves runs of 2^d consecutive words) instead of going through LDS.
constexpr bool ntt_direct(int d) { return d <= 1; }

__device__ __forceinline__ int lds_idx(int j) { return j + (j >> 5); }

// Group index of (thread, u) in a pass of D stages (G = 2^(EL - D) groups of 2^D registers per
// thread): the G groups of a thread are 64 apart and the 64 G groups of a wave are contiguous.
// A pass then keeps each wave on words [64 E w, 64 E (w + 1)) of the row (wave w, E = 2^EL) when
// its blocks of 2^(LOGN - S0) words have spans LOW = 2^(LOGN - S0 - D) dividing 64 G, that is
// when S0 >= LOGN - 6 - EL (wave_local); between two such passes a wave reads back only words it
// wrote itself, so it needs no workgroup barrier.
template <int EL, int D>
__device__ __forceinline__ int group_of(int tid, int u) {
  constexpr int G = 1 << (EL - D);
  return G == 1 ? tid : (tid >> 6) * 64 * G + u * 64 + (tid & 63);
}
template <int LOGN, int EL>
constexpr bool wave_local(int s0) { return s0 >= LOGN - 6 - EL; }
// Orders a wave's LDS writes before its later reads of words other lanes wrote.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LOGN, int EL, int S0, int D>
__device__ __forceinline__ int elem_index(int tid, int u, int m) {
  constexpr int N = 1 << LOGN, LOW = N >> (S0 + D);
  const int g = group_of<EL, D>(tid, u);
  return (g / LOW) * (N >> S0) + m * LOW + (g % LOW);
}
// lds_idx(elem_index(tid, u, m)) as a part that depends on the thread and u plus a compile-time
// offset for m, so that the 2^D accesses of a group share one address and differ in the offset
// field. With a = (g / LOW) 2^(LOGN - S0) and r = g mod LOW the index is a + m LOW + r, and its
// padding word count (index >> 5) splits into a >> 5, (m LOW) >> 5 and r >> 5: either a and m LOW
// are multiples of 32, or LOW < 32 divides 32 (then r < LOW adds no carry), or the block
// 2^(LOGN - S0) < 32 divides 32 (then nothing inside a block carries past a multiple of 32).
template <int LOGN, int EL, int S0, int D>
__device__ __forceinline__ int lds_base(int tid, int u) {
  constexpr int N = 1 << LOGN, LOW = N >> (S0 + D);
  const int g = group_of<EL, D>(tid, u);
  const int a = (g / LOW) * (N >> S0), r = g % LOW;
  return a + (a >> 5) + r + (r >> 5);
}
template <int LOGN, int S0, int D>
constexpr int lds_off(int m) {
  return m * ((1 << LOGN) >> (S0 + D)) + ((m * ((1 << LOGN) >> (S0 + D))) >> 5);
}

// Forward stages [S0, S0 + D) on 2^(EL - D) groups of 2^D registers.
template <int LOGN, int EL, int S0, int D>
__device__ __forceinline__ void fwd_pass(uint64_t* x, int tid, const uint64_t* __restrict__ W,
                                         const uint64_t* __restrict__ Wq, uint64_t p) {
  constexpr int N = 1 << LOGN, LOW = N >> (S0 + D), G = 1 << (EL - D);
  const uint64_t four_p = 4 * p;
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const int hi = group_of<EL, D>(tid, u) / LOW;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      const int half = 1 << (D - 1 - r);
#pragma unroll
      for (int blk = 0; blk < (1 << r); ++blk) {
        const int widx = (1 << (S0 + r)) + ((hi << r) | blk);
        const uint64_t w = W[widx], wq = Wq[widx];
#pragma unroll
        for (int m = 0; m < half; ++m) {
          const int a = u * (1 << D) + blk * 2 * half + m, b = a + half;
          const uint64_t U = x[a];
          const uint64_t V = shoup_lazy4(x[b], w, wq, p);
          x[a] = U + V;
          x[b] = U - V + four_p;
        }
      }
    }
  }
}

constexpr int ilog2(int v) { return v > 1 ? 1 + ilog2(v >> 1) : 0; }

// Inverse butterflies leave sums unreduced: a word is below 2^k 4p, where k counts the stages since
// its last Shoup product. Within a group of 2^D registers this depends only on the offset m: before
// the stage of span 2^j, k = j for m mod 2^j = 0 and otherwise j - 1 - floor(log2(m mod 2^j)).
constexpr int inv_bound(int j, int m) {
  return (m & ((1 << j) - 1)) == 0 ? j : j - 1 - ilog2(m & ((1 << j) - 1));
}

// Inverse stages S0 + D - 1 down to S0. With RED, every word is brought back below 4p at the end
// (k conditional subtractions for a word of bound exponent k); without, words may reach 2^D 4p.
template <int LOGN, int EL, int S0, int D, bool RED>
__device__ __forceinline__ void inv_pass(uint64_t* x, int tid, const uint64_t* __restrict__ W,
                                         const uint64_t* __restrict__ Wq, uint64_t p) {
  constexpr int N = 1 << LOGN, LOW = N >> (S0 + D), G = 1 << (EL - D);
  const uint64_t four_p = 4 * p;
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const int hi = group_of<EL, D>(tid, u) / LOW;
#pragma unroll
    for (int r = D - 1; r >= 0; --r) {
      const int half = 1 << (D - 1 - r);
#pragma unroll
      for (int blk = 0; blk < (1 << r); ++blk) {
        const int widx = (1 << (S0 + r)) + ((hi << r) | blk);
        const uint64_t w = W[widx], wq = Wq[widx];
#pragma unroll
        for (int m = 0; m < half; ++m) {
          const int a = u * (1 << D) + blk * 2 * half + m, b = a + half;
          const uint64_t U = x[a], V = x[b];
          x[a] = U + V;
          x[b] = shoup_lazy4(U - V + (four_p << inv_bound(D - 1 - r, m)), w, wq, p);
        }
      }
    }
    if constexpr (RED) {
#pragma unroll
      for (int m = 0; m < (1 << D); ++m) {
        uint64_t v = x[u * (1 << D) + m];
#pragma unroll
        for (int j = inv_bound(D, m) - 1; j >= 0; --j)
          if (v >= (four_p << j)) v -= four_p << j;
        x[u * (1 << D) + m] = v;
      }
    }
  }
}

// A thread writes back exactly the LDS words it read for the same pass, so a pass needs a barrier
// only before its reads.
template <int LOGN, int EL, int S0, int D, class V>
__device__ __forceinline__ void to_lds(V* lds, const V* x, int tid) {
#pragma unroll
  for (int u = 0; u < (1 << (EL - D)); ++u) {
    V* base = lds + lds_base<LOGN, EL, S0, D>(tid, u);
#pragma unroll
    for (int m = 0; m < (1 << D); ++m) base[lds_off<LOGN, S0, D>(m)] = x[u * (1 << D) + m];
  }
}
template <int LOGN, int EL, int S0, int D, class V>
__device__ __forceinline__ void from_lds(V* x, const V* lds, int tid) {
#pragma unroll
  for (int u = 0; u < (1 << (EL - D)); ++u) {
    const V* base = lds + lds_base<LOGN, EL, S0, D>(tid, u);
#pragma unroll
    for (int m = 0; m < (1 << D); ++m) x[u * (1 << D) + m] = base[lds_off<LOGN, S0, D>(m)];
  }
}

// Forward passes starting at stage S0 (> 0); the previous pass has left its outputs in LDS. With
// KEEP, the last pass leaves its outputs in registers.
template <int LOGN, int EL, int S0, bool KEEP>
__device__ __forceinline__ void fwd_passes(uint64_t* x, uint64_t* lds, int tid,
                                           const uint64_t* __restrict__ W,
                                           const uint64_t* __restrict__ Wq, uint64_t p) {
  constexpr int D = (LOGN - S0 < EL) ? LOGN - S0 : EL;
  // the previous pass (stages [S0 - EL, S0)) wrote what this one reads
  if constexpr (wave_local<LOGN, EL>(S0 - EL) && wave_local<LOGN, EL>(S0)) wave_sync();
  else __syncthreads();
  from_lds<LOGN, EL, S0, D>(x, lds, tid);
  fwd_pass<LOGN, EL, S0, D>(x, tid, W, Wq, p);
  if constexpr (S0 + D < LOGN) {
    to_lds<LOGN, EL, S0, D>(lds, x, tid);
    fwd_passes<LOGN, EL, S0 + D, KEEP>(x, lds, tid, W, Wq, p);
  } else if constexpr (!KEEP) {
    to_lds<LOGN, EL, S0, D>(lds, x, tid);
  }
}

// Inverse passes from pass K (stages [K EL, K EL + D)) down to pass 1; the inputs of pass K are
// in LDS. Pass 0 is left to the caller, which keeps its outputs in registers.
template <int LOGN, int EL, int K>
__device__ __forceinline__ void inv_passes(uint64_t* x, uint64_t* lds, int tid,
                                           const uint64_t* __restrict__ W,
                                           const uint64_t* __restrict__ Wq, uint64_t p) {
  constexpr int S0 = K * EL, D = (LOGN - S0 < EL) ? LOGN - S0 : EL;
  // the previous pass (stages from S0 + EL up) wrote what this one reads
  if constexpr (wave_local<LOGN, EL>(S0 + EL) && wave_local<LOGN, EL>(S0)) wave_sync();
  else __syncthreads();
  from_lds<LOGN, EL, S0, D>(x, lds, tid);
  inv_pass<LOGN, EL, S0, D, true>(x, tid, W, Wq, p);
  to_lds<LOGN, EL, S0, D>(lds, x, tid);
  if constexpr (K > 1) inv_passes<LOGN, EL, K - 1>(x, lds, tid, W, Wq, p);
}

template <NttLoad LD>
__device__ __forceinline__ uint64_t load_elem(const Consts& C, const void* in, size_t row, int nprimes, int N,
                                              int j, uint64_t p) {
  if constexpr (LD == LOAD_U64) {
    return static_cast<const uint64_t*>(in)[row * N + j];
  } else if constexpr (LD == LOAD_DIGITS) {
    // D_i = [c2_i (Q/q_i)^-1]_{q_i} < q_i < 2 q_j, reduced mod q_j = p by one subtraction
    const int L = nprimes;
    const int i = (int)((row / L) % L);
    const size_t unit = row / ((size_t)L * L);
    const uint64_t v = static_cast<const uint64_t*>(in)[(unit * L + i) * N + j];
    const uint64_t d = shoup(v, C.qhat_inv[i], C.qhat_inv_shoup[i], C.prm[i].p);
    return d >= p ? d - p : d;
  } else if constexpr (LD == LOAD_LIFT_T) {
    const uint32_t v = static_cast<const uint32_t*>(in)[(row / nprimes) * N + j];
    return v <= (PEPSI_T - 1) / 2 ? (uint64_t)v : p - (uint64_t)(PEPSI_T - v);
  } else if constexpr (LD == LOAD_I8) {
    const int v = static_cast<const int8_t*>(in)[(row / nprimes) * N + j];
    return v >= 0 ? (uint64_t)v : p - (uint64_t)(-v);
  } else {
    const int v = static_cast<const int32_t*>(in)[(row / nprimes) * N + j];
    return v >= 0 ? (uint64_t)v : p - (uint64_t)(-(int64_t)v);
  }
}

// Output word j of row `row` of the forward transform: reduced from [0, 57p) and stored whole, or
// split 27/27 at its place in a plaintext store.
template <NttStore ST>
__device__ __forceinline__ void store_elem(void* out, size_t row, int N, int nprimes, const PtLayout& pl, int j,
                                           uint64_t v, uint64_t p64, uint64_t p) {
  v = shoup_lazy(v, 1, p64, p);   // [0, 57p) -> [0, 2p)
  if (v >= p) v -= p;
  if constexpr (ST == STORE_U64) {
    static_cast<uint64_t*>(out)[row * N + j] = v;
  } else {
    const size_t l = row % nprimes, jb = row / nprimes, cj = jb % pl.ell, b = jb / pl.ell + pl.bbase;
    const size_t G = b / pl.gs, g = b % pl.gs;
    const size_t at = ((((G * pl.ell + cj) * nprimes + l) * (N / PT_BLOCK) + j / PT_BLOCK) * pl.gs + g) * PT_BLOCK +
                      j % PT_BLOCK;
    static_cast<uint64_t*>(out)[at] = (v & ((1ull << 27) - 1)) | ((v >> 27) << 32);
  }
}

template <int LOGN, NttLoad LD, NttStore ST, int EL = ntt_el<LOGN>()>
__global__ void __launch_bounds__((1 << LOGN) >> EL)
k_ntt_fwd(Tables T, const void* __restrict__ in, void* __restrict__ out, int nprimes, int first, PtLayout pl) {
  constexpr int N = 1 << LOGN, E = 1 << EL, TT = N >> EL;
  constexpr int SL = (LOGN - 1) / EL * EL, DL = LOGN - SL;   // last pass: stages [SL, LOGN)
  constexpr bool KEEP = ntt_direct(DL);
  __shared__ uint64_t lds[N + N / 32];
  const size_t row = blockIdx.x;
  const int pidx = first + (int)(row % nprimes);
  const uint64_t p = T.c->prm[pidx].p;
  const uint64_t* W = T.psi_rev + (size_t)pidx * N;
  const uint64_t* Wq = T.psi_rev_shoup + (size_t)pidx * N;
  const int tid = threadIdx.x;
  uint64_t x[E];
#pragma unroll
  for (int m = 0; m < E; ++m) x[m] = load_elem<LD>(*T.c, in, row, nprimes, N, m * TT + tid, p);
  fwd_pass<LOGN, EL, 0, EL>(x, tid, W, Wq, p);
  to_lds<LOGN, EL, 0, EL>(lds, x, tid);
  fwd_passes<LOGN, EL, EL, KEEP>(x, lds, tid, W, Wq, p);
  const uint64_t p64 = T.c->prm[pidx].barrett >> 52;     // floor(2^64 / p)
  if constexpr (KEEP) {
    // Each thread holds runs of 2^DL consecutive outputs.
#pragma unroll
    for (int u = 0; u < (1 << (EL - DL)); ++u)
#pragma unroll
      for (int m = 0; m < (1 << DL); ++m)
        store_elem<ST>(out, row, N, nprimes, pl, elem_index<LOGN, EL, SL, DL>(tid, u, m), x[u * (1 << DL) + m],
                       p64, p);
  } else {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int j = m * TT + tid;
      store_elem<ST>(out, row, N, nprimes, pl, j, lds[lds_idx(j)], p64, p);
    }
  }
}

// Where an inverse transform's input words come from: a plain row, or a component of a
// ciphertext product over Q u B formed on the fly (InvProducts).  The row's unit, component and
// prime are uniform over the workgroup.
struct InvSrc { const uint64_t* xq; const uint64_t* xb; const TensorJob* jobs; };
template <int IL>
struct InvRow {
  const uint64_t* in;
  size_t row;
  // product rows: the operands' limb rows and the constants added to c0
  const uint64_t *x0, *x1, *y0, *y1;
  uint64_t ax, ay;
  int comp;
  Prime pr;
  __device__ __forceinline__ InvRow(const Consts& C, const uint64_t* in_, size_t row_, const InvSrc& src, int N)
      : in(in_), row(row_) {
    if constexpr (IL != 0) {
      const int L = C.L, K = C.K, P = L + K;
      const int p = (int)(row % P);
      comp = (int)((row / P) % 3);
      const size_t unit = row / ((size_t)3 * P);
      pr = C.prm[p];
      ax = ay = 0;
      if constexpr (IL == INV_SQUARES) {
        const uint64_t* base = p < L ? src.xq + (unit * 2 * L + p) * N : src.xb + (unit * 2 * K + (p - L)) * N;
        const size_t cstep = (size_t)(p < L ? L : K) * N;
        x0 = y0 = base;
        x1 = y1 = base + cstep;
      } else {
        const TensorJob J = src.jobs[unit];
        const size_t a0 = p < L ? (size_t)p * N : (size_t)(p - L) * N;
        const size_t cstep = (size_t)(p < L ? L : K) * N;
        const uint64_t* xs = p < L ? J.xq : J.xb;
        const uint64_t* ys = p < L ? J.yq : J.yb;
        x0 = xs + a0; x1 = xs + a0 + cstep;
        y0 = ys + a0; y1 = ys + a0 + cstep;
        if (J.ax) ax = J.ax[p];
        if (J.ay) ay = J.ay[p];
      }
    }
  }
  // The first inverse pass takes words below 4p, so the products are reduced lazily (below 3p),
  // and each component loads only the operand rows it uses.
  __device__ __forceinline__ uint64_t at(int N, int j) const {
    if constexpr (IL == 0) {
      return in[row * N + j];
    } else if constexpr (IL == INV_SQUARES) {
      if (comp == 0) {
        const uint64_t a = x0[j];
        return mulmod_lazy(a, a, pr);
      }
      if (comp == 2) {
        const uint64_t b = x1[j];
        return mulmod_lazy(b, b, pr);
      }
      const uint64_t a = x0[j];
      return mulmod_lazy(a + a, x1[j], pr);            // 2a < 2p: the product is below 2^109
    } else {
      if (comp == 2) return mulmod_lazy(x1[j], y1[j], pr);
      const uint64_t a = ax ? addmod(x0[j], ax, pr.p) : x0[j];
      const uint64_t c = ay ? addmod(y0[j], ay, pr.p) : y0[j];
      if (comp == 0) return mulmod_lazy(a, c, pr);
      const u128 m = (u128)a * y1[j] + (u128)x1[j] * c;
      return reduce116_lazy((uint64_t)m, (uint64_t)(m >> 64), pr);
    }
  }
};

template <int LOGN, int IL = 0, int EL = ntt_el<LOGN>()>
__global__ void __launch_bounds__((1 << LOGN) >> EL) __attribute__((amdgpu_waves_per_eu(ntt_waves<EL>())))
k_ntt_inv(Tables T, const uint64_t* __restrict__ in, uint64_t* __restrict__ out, int nprimes, int first, InvSrc src) {
  constexpr int N = 1 << LOGN, E = 1 << EL, TT = N >> EL, NP = (LOGN + EL - 1) / EL;
  constexpr int SL = (NP - 1) * EL, DL = LOGN - SL;   // first inverse pass: stages [SL, LOGN)
  __shared__ uint64_t lds[N + N / 32];
  const size_t row = blockIdx.x;
  const int pidx = first + (int)(row % nprimes);
  const uint64_t p = T.c->prm[pidx].p;
  const uint64_t* W = T.ipsi_rev + (size_t)pidx * N;
  const uint64_t* Wq = T.ipsi_rev_shoup + (size_t)pidx * N;
  const int tid = threadIdx.x;
  const InvRow<IL> src_row(*T.c, in, row, src, N);
  uint64_t x[E];
  if constexpr (ntt_direct(DL) && NP > 2) {
    // Runs of 2^DL consecutive inputs go straight to registers for the first pass.
#pragma unroll
    for (int u = 0; u < (1 << (EL - DL)); ++u)
#pragma unroll
      for (int m = 0; m < (1 << DL); ++m)
        x[u * (1 << DL) + m] = src_row.at(N, elem_index<LOGN, EL, SL, DL>(tid, u, m));
    inv_pass<LOGN, EL, SL, DL, true>(x, tid, W, Wq, p);
    to_lds<LOGN, EL, SL, DL>(lds, x, tid);
    inv_passes<LOGN, EL, NP - 2>(x, lds, tid, W, Wq, p);
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int j = m * TT + tid;
      lds[lds_idx(j)] = src_row.at(N, j);
    }
    __syncthreads();   // written in row order, read by the first pass's groups
    inv_passes<LOGN, EL, NP - 1>(x, lds, tid, W, Wq, p);
  }
  __syncthreads();
  from_lds<LOGN, EL, 0, EL>(x, lds, tid);
  inv_pass<LOGN, EL, 0, EL, false>(x, tid, W, Wq, p);
  const uint64_t ni = T.c->n_inv[pidx], niq = T.c->n_inv_shoup[pidx];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int j = m * TT + tid;
    out[row * N + j] = shoup(x[m], ni, niq, p);
  }
}

// ---------------- transforms over t ----------------

__device__ __forceinline__ int brv(int k, int logn) { return (int)(__brev((unsigned)k) >> (32 - logn)); }

template <int LOGN>
__device__ void ntt_t_lds(uint32_t* a, const uint32_t* __restrict__ w_rev) {
  constexpr int N = 1 << LOGN;
  for (int s = 0; s < LOGN; ++s) {
    const int t = N >> (s + 1);
    for (int bi = threadIdx.x; bi < N / 2; bi += blockDim.x) {
      const int i = bi / t, off = bi % t;
      const int x = i * 2 * t + off, y = x + t;
      const uint32_t w = w_rev[(1 << s) + i];
      const uint32_t U = a[x], V = mulmod_t(a[y], w);
      a[x] = addmod_t(U, V);
      a[y] = submod_t(U, V);
    }
    __syncthreads();
  }
}

template <int LOGN>
__global__ void __launch_bounds__(256) k_decode(Tables T, const uint32_t* __restrict__ poly,
                                               uint32_t* __restrict__ slots) {
  constexpr int N = 1 << LOGN;
  __shared__ uint32_t a[N];
  const size_t row = blockIdx.x;
  for (int k = threadIdx.x; k < N; k += blockDim.x) a[k] = poly[row * N + k] % PEPSI_T;
  __syncthreads();
  ntt_t_lds<LOGN>(a, T.psit_rev);
  for (int k = threadIdx.x; k < N; k += blockDim.x) slots[row * N + brv(k, LOGN)] = a[k];
}

// a b mod t for t = 2^16 + 1 and a, b <= 2^16: with a b = xh 2^16 + xl and 2^16 = -1 mod t, the
// residue is xl - xh.
__device__ __forceinline__ uint32_t mulmod_t16(uint32_t a, uint32_t b) {
  const uint64_t x = (uint64_t)a * b;   // <= 2^32
  const uint32_t xl = (uint32_t)x & 0xffffu, xh = (uint32_t)(x >> 16);
  return xl >= xh ? xl - xh : xl + PEPSI_T - xh;
}

// Inverse stages S0 + D - 1 down to S0 over Z_t (Gentleman-Sande, residues kept reduced), with the
// register layout of inv_pass.
template <int LOGN, int EL, int S0, int D>
__device__ __forceinline__ void inv_pass_t(uint32_t* x, int tid, const uint32_t* __restrict__ W) {
  constexpr int N = 1 << LOGN, LOW = N >> (S0 + D), G = 1 << (EL - D);
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const int hi = group_of<EL, D>(tid, u) / LOW;
#pragma unroll
    for (int r = D - 1; r >= 0; --r) {
      const int half = 1 << (D - 1 - r);
#pragma unroll
      for (int blk = 0; blk < (1 << r); ++blk) {
        const uint32_t w = W[(1 << (S0 + r)) + ((hi << r) | blk)];
#pragma unroll
        for (int m = 0; m < half; ++m) {
          const int a = u * (1 << D) + blk * 2 * half + m, b = a + half;
          const uint32_t U = x[a], V = x[b];
          x[a] = addmod_t(U, V);
          x[b] = mulmod_t16(submod_t(U, V), w);
        }
      }
    }
  }
}
template <int LOGN, int EL, int K>
__device__ __forceinline__ void inv_passes_t(uint32_t* x, uint32_t* lds, int tid, const uint32_t* __restrict__ W) {
  constexpr int S0 = K * EL, D = (LOGN - S0 < EL) ? LOGN - S0 : EL;
  __syncthreads();
  from_lds<LOGN, EL, S0, D>(x, lds, tid);
  inv_pass_t<LOGN, EL, S0, D>(x, tid, W);
  to_lds<LOGN, EL, S0, D>(lds, x, tid);
  if constexpr (K > 1) inv_passes_t<LOGN, EL, K - 1>(x, lds, tid, W);
}

// Inverse transform over t of a row whose bit-reversed evaluations are in LDS (at lds_idx
// positions), scaled by N^-1: coefficient m TT + tid ends in x[m].
template <int LOGN, int EL>
__device__ __forceinline__ void intt_t_row(uint32_t* x, uint32_t* lt, int tid, const Tables& T) {
  constexpr int E = 1 << EL, NP = (LOGN + EL - 1) / EL;
  static_assert(NP >= 2, "at least two passes");
  inv_passes_t<LOGN, EL, NP - 1>(x, lt, tid, T.ipsit_rev);
  __syncthreads();
  from_lds<LOGN, EL, 0, EL>(x, lt, tid);
  inv_pass_t<LOGN, EL, 0, EL>(x, tid, T.ipsit_rev);
  const uint32_t ninv = T.c->n_inv_t;
#pragma unroll
  for (int m = 0; m < E; ++m) x[m] = mulmod_t16(x[m], ninv);
}

// Row (b, j): slot s is 1 iff position j is one of the h codeword positions of bin s; the row is
// then inverse-transformed over t (bit-reversed slots in, coefficients out) and scaled by N^-1.
// Same register passes as k_ntt_inv: each thread reads the codewords of E slots (coalesced) and
// places their bits at the bit-reversed LDS positions; the last pass leaves coefficient m TT + tid
// in register m.
template <int LOGN, int EL = ntt_t_el<LOGN>()>
__global__ void __launch_bounds__((1 << LOGN) >> EL)
k_encode_planes(Tables T, const uint16_t* __restrict__ cw, int h, int ell, int b0, uint32_t* __restrict__ poly) {
  constexpr int N = 1 << LOGN, E = 1 << EL, TT = N >> EL;
  __shared__ uint32_t lt[N + N / 32];
  const size_t row = blockIdx.x;
  const int b = (int)(row / ell) + b0, j = (int)(row % ell);
  const uint16_t* base = cw + (size_t)b * N * h;
  const int tid = threadIdx.x;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int s = m * TT + tid;
    uint32_t y = 0;
    for (int r = 0; r < h; ++r) y |= (base[(size_t)s * h + r] == j) ? 1u : 0u;
    lt[lds_idx(brv(s, LOGN))] = y;
  }
  uint32_t x[E];
  intt_t_row<LOGN, EL>(x, lt, tid, T);
#pragma unroll
  for (int m = 0; m < E; ++m) poly[row * N + m * TT + tid] = x[m];
}

// Batch encoding of slot rows (slot s of row r at slots[r N + s]): the bit-reversed slots are
// inverse-transformed over t like the bit planes of k_encode_planes.
template <int LOGN, int EL = ntt_t_el<LOGN>()>
__global__ void __launch_bounds__((1 << LOGN) >> EL)
k_encode(Tables T, const uint32_t* __restrict__ slots, uint32_t* __restrict__ poly) {
  constexpr int N = 1 << LOGN, E = 1 << EL, TT = N >> EL;
  __shared__ uint32_t lt[N + N / 32];
  const size_t row = blockIdx.x;
  const int tid = threadIdx.x;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int s = m * TT + tid;
    lt[lds_idx(brv(s, LOGN))] = slots[row * N + s] % PEPSI_T;
  }
  uint32_t x[E];
  intt_t_row<LOGN, EL>(x, lt, tid, T);
#pragma unroll
  for (int m = 0; m < E; ++m) poly[row * N + m * TT + tid] = x[m];
}

template <int LOGN>
void launch_fwd(const Tables& T, const void* in, NttLoad ld, void* out, NttStore st, int rows,
                int nprimes, int first, const PtLayout& pl, hipStream_t s) {
  const dim3 grid(rows), block((1 << LOGN) >> ntt_el<LOGN>());
#define PEPSI_FWD(L_, S_) hipLaunchKernelGGL((k_ntt_fwd<LOGN, L_, S_>), grid, block, 0, s, T, in, out, nprimes, first, pl)
  if (st == STORE_U64) {
    switch (ld) {
      case LOAD_U64: PEPSI_FWD(LOAD_U64, STORE_U64); break;
      case LOAD_LIFT_T: PEPSI_FWD(LOAD_LIFT_T, STORE_U64); break;
      case LOAD_I8: PEPSI_FWD(LOAD_I8, STORE_U64); break;
      case LOAD_I32: PEPSI_FWD(LOAD_I32, STORE_U64); break;
      case LOAD_DIGITS: PEPSI_FWD(LOAD_DIGITS, STORE_U64); break;
    }
  } else {
    if (ld == LOAD_LIFT_T) PEPSI_FWD(LOAD_LIFT_T, STORE_PLAINTEXT);
  }
#undef PEPSI_FWD
}

}  // namespace

void ntt_forward(const Tables& T, int logn, const void* in, NttLoad load, void* out, NttStore store,
                 int rows, int nprimes, int first, hipStream_t s) {
  if (rows <= 0) return;
  switch (logn) {
    case 10: launch_fwd<10>(T, in, load, out, store, rows, nprimes, first, PtLayout{}, s); break;
    case 11: launch_fwd<11>(T, in, load, out, store, rows, nprimes, first, PtLayout{}, s); break;
    case 12: launch_fwd<12>(T, in, load, out, store, rows, nprimes, first, PtLayout{}, s); break;
    case 13: launch_fwd<13>(T, in, load, out, store, rows, nprimes, first, PtLayout{}, s); break;
    case 14: launch_fwd<14>(T, in, load, out, store, rows, nprimes, first, PtLayout{}, s); break;
  }
}

void ntt_forward_plaintexts(const Tables& T, int logn, const uint32_t* in, uint64_t* out, int nb, int L,
                            const PtLayout& pl, hipStream_t s) {
  const int rows = nb * pl.ell * L;
  if (rows <= 0) return;
  switch (logn) {
    case 10: launch_fwd<10>(T, in, LOAD_LIFT_T, out, STORE_PLAINTEXT, rows, L, 0, pl, s); break;
    case 11: launch_fwd<11>(T, in, LOAD_LIFT_T, out, STORE_PLAINTEXT, rows, L, 0, pl, s); break;
    case 12: launch_fwd<12>(T, in, LOAD_LIFT_T, out, STORE_PLAINTEXT, rows, L, 0, pl, s); break;
    case 13: launch_fwd<13>(T, in, LOAD_LIFT_T, out, STORE_PLAINTEXT, rows, L, 0, pl, s); break;
    case 14: launch_fwd<14>(T, in, LOAD_LIFT_T, out, STORE_PLAINTEXT, rows, L, 0, pl, s); break;
  }
}

template <int IL>
void launch_inv(const Tables& T, int logn, const uint64_t* in, uint64_t* out, int rows, int nprimes, int first,
                const InvSrc& src, hipStream_t s) {
#define PEPSI_INV(LL) hipLaunchKernelGGL((k_ntt_inv<LL, IL>), dim3(rows), dim3((1 << LL) >> ntt_el<LL>()), 0, s, T, in, \
                                         out, nprimes, first, src)
  switch (logn) {
    case 10: PEPSI_INV(10); break;
    case 11: PEPSI_INV(11); break;
    case 12: PEPSI_INV(12); break;
    case 13: PEPSI_INV(13); break;
    case 14: PEPSI_INV(14); break;
  }
#undef PEPSI_INV
}

void ntt_inverse(const Tables& T, int logn, const uint64_t* in, uint64_t* out, int rows, int nprimes,
                 int first, hipStream_t s) {
  if (rows <= 0) return;
  launch_inv<0>(T, logn, in, out, rows, nprimes, first, InvSrc{nullptr, nullptr, nullptr}, s);
}

void ntt_inverse_products(const Tables& T, int logn, InvProducts mode, const uint64_t* xq, const uint64_t* xb,
                          const TensorJob* jobs, uint64_t* out, int units, int nprimes, hipStream_t s) {
  const int rows = units * 3 * nprimes;
  if (rows <= 0) return;
  if (mode == INV_SQUARES)
    launch_inv<INV_SQUARES>(T, logn, nullptr, out, rows, nprimes, 0, InvSrc{xq, xb, nullptr}, s);
  else
    launch_inv<INV_TENSOR>(T, logn, nullptr, out, rows, nprimes, 0, InvSrc{nullptr, nullptr, jobs}, s);
}

#define PEPSI_T_DISPATCH(KERNEL, ...)                                                          \
  switch (logn) {                                                                              \
    case 10: hipLaunchKernelGGL(KERNEL<10>, dim3(rows), dim3(256), 0, s, __VA_ARGS__); break;  \
    case 11: hipLaunchKernelGGL(KERNEL<11>, dim3(rows), dim3(256), 0, s, __VA_ARGS__); break;  \
    case 12: hipLaunchKernelGGL(KERNEL<12>, dim3(rows), dim3(256), 0, s, __VA_ARGS__); break;  \
    case 13: hipLaunchKernelGGL(KERNEL<13>, dim3(rows), dim3(256), 0, s, __VA_ARGS__); break;  \
    case 14: hipLaunchKernelGGL(KERNEL<14>, dim3(rows), dim3(256), 0, s, __VA_ARGS__); break;  \
  }

void encode_slots(const Tables& T, int logn, const uint32_t* slots, uint32_t* poly, int rows,
                  hipStream_t s) {
  if (rows <= 0) return;
#define PEPSI_ENC1(LL) hipLaunchKernelGGL(k_encode<LL>, dim3(rows), dim3((1 << LL) >> ntt_t_el<LL>()), 0, s, T, slots, \
                                          poly)
  switch (logn) {
    case 10: PEPSI_ENC1(10); break;
    case 11: PEPSI_ENC1(11); break;
    case 12: PEPSI_ENC1(12); break;
    case 13: PEPSI_ENC1(13); break;
    case 14: PEPSI_ENC1(14); break;
  }
#undef PEPSI_ENC1
}
void decode_slots(const Tables& T, int logn, const uint32_t* poly, uint32_t* slots, int rows,
                  hipStream_t s) {
  if (rows <= 0) return;
  PEPSI_T_DISPATCH(k_decode, T, poly, slots)
}
void encode_server_planes(const Tables& T, int logn, const uint16_t* cw, int h, int ell, int b0,
                          int nb, uint32_t* poly, hipStream_t s) {
  const int rows = nb * ell;
  if (rows <= 0) return;
#define PEPSI_ENC(LL) hipLaunchKernelGGL(k_encode_planes<LL>, dim3(rows), dim3((1 << LL) >> ntt_t_el<LL>()), 0, s, T, \
                                         cw, h, ell, b0, poly)
  switch (logn) {
    case 10: PEPSI_ENC(10); break;
    case 11: PEPSI_ENC(11); break;
    case 12: PEPSI_ENC(12); break;
    case 13: PEPSI_ENC(13); break;
    case 14: PEPSI_ENC(14); break;
  }
#undef PEPSI_ENC
}

}  // namespace pepsi
