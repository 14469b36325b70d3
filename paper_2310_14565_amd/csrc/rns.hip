// RNS kernels of the BFV evaluation: exact base extension, the exact
// ciphertext-product rescale round(t d / Q), relinearisation with the RNS
// gadget, the select-and-sum of the server computation, and elementwise steps.
//
// Exactness.  A centred base extension needs v = round(sum_i y_i / q_i) and
// the rescale needs R = round(sum_i y_i theta_i).  v is at most the number of
// terms and is computed in double precision with a proven error below 2^-45;
// R can be large and is computed in 64.64 fixed point with an error below
// n 2^-41.  When the fraction lies within that bound (with margin) of 1/2 the
// coefficient takes the exact path (crt_exact: the integer is rebuilt in
// multiword arithmetic and compared with half the modulus), so every output
// equals the textbook integer result.
#include "kernels.hpp"

#include <algorithm>

namespace pepsi {
namespace {

constexpr int TPB = 256;

struct FixAcc { uint64_t ip, frac; };

// a += y * C, C = floor(c 2^128) with c in [0, 1): keeps the integer part and the top 64
// fraction bits; the dropped low word and the truncation of C cost < 2^-64 + 2^-74 per term.
__device__ __forceinline__ void fix_add(FixAcc& a, uint64_t y, const Fix128& C) {
  const uint64_t p0h = mulhi64(y, C.lo);
  const uint64_t p1l = y * C.hi, p1h = mulhi64(y, C.hi);
  const uint64_t w1 = p0h + p1l;
  const uint64_t w2 = p1h + (w1 < p0h ? 1 : 0);
  const uint64_t f = a.frac + w1;
  a.ip += w2 + (f < w1 ? 1 : 0);
  a.frac = f;
}
// round(S) for S in [A, A + (n + 1) 2^-64): floor(A + 1/2), flagged when S may round higher.
__device__ __forceinline__ uint64_t fix_round(const FixAcc& a, int nterms, bool* ambiguous) {
  const uint64_t f = a.frac + (1ull << 63);
  const uint64_t carry = f < a.frac ? 1 : 0;
  *ambiguous = f > ~0ull - 2ull * (uint64_t)(nterms + 2);
  return a.ip + carry;
}

// The theta sum of the rescale with C read to 96 bits: y = y1 2^32 + y0 (y < 2^54) and C's top
// words t2, t1, t0 at 2^-32, 2^-64 and 2^-96.  In units of 2^-64 the product is
//   y1 t2 2^64 + (y0 t2 + y1 t1) 2^32 + (y0 t1 + y1 t0) + y0 t0 2^-32;
// the low half of the last term and C beyond 96 bits are dropped, so each term is less than
// 2^22 + 2 units short.
__device__ __forceinline__ void fix_add96(FixAcc& a, uint64_t y, const Fix128& C) {
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  const uint32_t t2 = (uint32_t)(C.hi >> 32), t1 = (uint32_t)C.hi, t0 = (uint32_t)(C.lo >> 32);
  const u128 m1 = (u128)((uint64_t)y0 * t2) + (uint64_t)y1 * t1;
  const u128 m0 = (u128)((uint64_t)y0 * t1) + (uint64_t)y1 * t0 + (((uint64_t)y0 * t0) >> 32);
  const u128 tot = m0 + (m1 << 32) + ((u128)((uint64_t)y1 * t2) << 64);
  const uint64_t f = a.frac + (uint64_t)tot;
  a.ip += (uint64_t)(tot >> 64) + (f < a.frac ? 1 : 0);
  a.frac = f;
}
// round(S) for S in [A, A + nterms (2^22 + 2) 2^-64): floor(A + 1/2), flagged when S may round
// higher.
__device__ __forceinline__ uint64_t fix_round96(const FixAcc& a, int nterms, bool* ambiguous) {
  const uint64_t f = a.frac + (1ull << 63);
  const uint64_t carry = f < a.frac ? 1 : 0;
  *ambiguous = f > ~0ull - ((uint64_t)(nterms + 1) << 23);
  return a.ip + carry;
}

// v = round(sum_i y_i / m_i) for y_i < m_i (the centring count of a base extension, v <= n), in
// double precision.  y_i converts with one rounding and 1/m_i is stored correctly rounded from
// the rounded m_i, so each product is within 3.01 2^-53 of y_i / m_i < 1; each fused addition
// adds at most i 2^-53, and the + 1/2 at most (n + 1) 2^-53.  For n <= 9 the total is below
// 2^-45, so outside a guard band of 2^-36 around the half-integers the rounding is the exact
// one; inside it *ambiguous is set.
template <int n>
__device__ __forceinline__ uint64_t round_fp(const uint64_t* y, const double* inv, bool* ambiguous) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < n; ++i) {
    const double yd = fma((double)(uint32_t)(y[i] >> 32), 0x1p32, (double)(uint32_t)y[i]);
    s = fma(yd, inv[i], s);
  }
  const double r = s + 0.5, f = floor(r), fr = r - f;
  *ambiguous = fr < 0x1p-36 || fr > 1.0 - 0x1p-36;
  return (uint64_t)f;
}

// Exact CRT: X = sum_k y_k * hat_k reduced into [0, M) by v subtractions of M.
// Returns v; *gt = (2 X > M); X is written to xout when given.
// The rare path of the kernels' roundings, inlined into them with its loops rolled: as a call it
// would make every caller keep its live values in callee-saved registers.  (X is an ordinary
// local array: a volatile one, kept in scratch memory, would count as a write to any memory, and
// the constants the callers read after it would then come through vector loads into many
// registers instead of scalar ones.)
__device__ __forceinline__ int crt_exact(const uint64_t* y, int cnt, const MWord* hat, const MWord& M,
                                      bool* gt, uint64_t* xout) {
  uint64_t X[PEPSI_MW];
#pragma unroll 1
  for (int w = 0; w < PEPSI_MW; ++w) X[w] = 0;
#pragma unroll 1
  for (int k = 0; k < cnt; ++k) {
    uint64_t carry = 0;
#pragma unroll 1
    for (int w = 0; w < PEPSI_MW; ++w) {
      const u128 t = (u128)y[k] * hat[k].w[w] + X[w] + carry;
      X[w] = (uint64_t)t;
      carry = (uint64_t)(t >> 64);
    }
  }
  int v = 0;
  for (;;) {
    bool ge = true;                               // X >= M ?
#pragma unroll 1
    for (int w = PEPSI_MW - 1; w >= 0; --w) {
      if (X[w] != M.w[w]) { ge = X[w] > M.w[w]; break; }
    }
    if (!ge) break;
    uint64_t borrow = 0;
#pragma unroll 1
    for (int w = 0; w < PEPSI_MW; ++w) {
      const u128 d = (u128)X[w] - M.w[w] - borrow;
      X[w] = (uint64_t)d;
      borrow = (uint64_t)(d >> 64) & 1;
    }
    ++v;
  }
  // 2X > M ?
  bool g = false;
#pragma unroll 1
  for (int w = PEPSI_MW - 1; w >= 0; --w) {
    const uint64_t x2 = (X[w] << 1) | (w > 0 ? X[w - 1] >> 63 : 0);
    const uint64_t top = w == PEPSI_MW - 1 ? (X[w] >> 63) : 0;   // bit shifted out of the top word
    if (top) { g = true; break; }
    if (x2 != M.w[w]) { g = x2 > M.w[w]; break; }
  }
  *gt = g;
  if (xout)
#pragma unroll 1
    for (int w = 0; w < PEPSI_MW; ++w) xout[w] = X[w];
  return v;
}

// Adds a kernel's count of exact-path coefficients to the device counter (when there is one).
__device__ __forceinline__ void count_exact(uint32_t* fallback, uint32_t nexact) {
  if (fallback && nexact) atomicAdd(fallback, nexact);
}

// Exact v = round(sum_i y_i / m_i) over Q (resp. B): the rare path of a centred extension.
// Each use adds 1 to nexact; a kernel adds its count to the device counter once, after its last
// store.  (An atomic on the way would make the compiler assume the constants read after it may
// have changed: it would then read them with vector loads into many registers, not into
// scalar ones.)
template <int L>
__device__ __forceinline__ uint64_t exact_round_q(const Consts& C, const uint64_t* yr, uint32_t& nexact) {
  uint64_t y[L];
  for (int i = 0; i < L; ++i) y[i] = yr[i];
  bool gt;
  const uint64_t v = (uint64_t)crt_exact(y, L, C.qhat_w, C.Qw, &gt, nullptr) + (gt ? 1 : 0);
  ++nexact;
  return v;
}
template <int K>
__device__ __forceinline__ uint64_t exact_round_b(const Consts& C, const uint64_t* yr, uint32_t& nexact) {
  uint64_t y[K];
  for (int j = 0; j < K; ++j) y[j] = yr[j];
  bool gt;
  const uint64_t v = (uint64_t)crt_exact(y, K, C.bhat_w, C.Bw, &gt, nullptr) + (gt ? 1 : 0);
  ++nexact;
  return v;
}

// Sums of products of residues below 2^54, without 128-bit carries: a = a1 2^27 + a0 and
// w = w1 2^27 + w0 give a w = a0 w0 + (a0 w1 + a1 w0) 2^27 + a1 w1 2^54, and the middle term is
// (a0 + a1)(w0 + w1) - a0 w0 - a1 w1 (Karatsuba), so three 64-bit accumulators of 32 x 32-bit
// products hold a sum of up to 16 products exactly (each term below 2^56).  The splits of the
// wave-uniform constants w stay on the scalar unit.
struct Split27 { uint32_t lo, hi, s; };
__device__ __forceinline__ Split27 split27(uint64_t x) {
  Split27 r;
  r.lo = (uint32_t)(x & ((1ull << 27) - 1));
  r.hi = (uint32_t)(x >> 27);
  r.s = r.lo + r.hi;
  return r;
}
struct Acc3 {
  uint64_t lo = 0, ms = 0, hi = 0;
  __device__ __forceinline__ void mac(const Split27& a, uint64_t w) {
    const uint32_t w0 = (uint32_t)(w & ((1ull << 27) - 1)), w1 = (uint32_t)(w >> 27);
    lo += (uint64_t)a.lo * w0;
    hi += (uint64_t)a.hi * w1;
    ms += (uint64_t)a.s * (w0 + w1);
  }
  // adds a plain integer (below 2^60 here) to the value, not to the middle term
  __device__ __forceinline__ void add(uint64_t v) { lo += v; ms += v; }
  __device__ __forceinline__ uint64_t reduce(const Prime& pr) const {
    const uint64_t mid = ms - lo - hi;
    const u128 v = (u128)lo + ((u128)mid << 27) + ((u128)hi << 54);   // below 2^112
    return reduce116((uint64_t)v, (uint64_t)(v >> 64), pr);
  }
  // congruent and below 3p, for a value that goes straight into a Shoup product
  __device__ __forceinline__ uint64_t reduce_lazy(const Prime& pr) const {
    const uint64_t mid = ms - lo - hi;
    const u128 v = (u128)lo + ((u128)mid << 27) + ((u128)hi << 54);
    return reduce116_lazy((uint64_t)v, (uint64_t)(v >> 64), pr);
  }
};

// Centred lift of x (residues mod q_0..q_{L-1}) into the residues mod b_0..b_{K-1}, K = L + 1.
template <int L>
__device__ __forceinline__ void ext_one(const Consts& C, const uint64_t* x, uint64_t* out,
                                        uint32_t& nexact) {
  constexpr int K = L + 1;
  uint64_t y[L];
#pragma unroll
  for (int i = 0; i < L; ++i) y[i] = shoup(x[i], C.qhat_inv[i], C.qhat_inv_shoup[i], C.prm[i].p);
  bool amb;
  uint64_t v = round_fp<L>(y, C.inv_q_d, &amb);
  Split27 ys[L];
#pragma unroll
  for (int i = 0; i < L; ++i) ys[i] = split27(y[i]);
  if (amb) v = exact_round_q<L>(C, y, nexact);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const Prime& P = C.prm[L + j];
    Acc3 acc;
    acc.mac(split27(v), P.p - C.q_mod_b[j]);
#pragma unroll
    for (int i = 0; i < L; ++i) acc.mac(ys[i], C.qhat_mod_b[i][j]);
    out[j] = acc.reduce(P);
  }
}

template <int L>
__global__ void __launch_bounds__(TPB) k_ext_q_to_b(Tables T, const uint64_t* __restrict__ in,
                                                   uint64_t* __restrict__ out, long ostride,
                                                   uint32_t* fallback) {
  const Consts& C = *T.c;
  constexpr int K = L + 1;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const size_t row = blockIdx.y;
  if (k >= N) return;
  uint64_t x[L], o[K];
#pragma unroll
  for (int i = 0; i < L; ++i) x[i] = in[(row * L + i) * N + k];
  uint32_t nexact = 0;
  ext_one<L>(C, x, o, nexact);
#pragma unroll
  for (int j = 0; j < K; ++j) out[row * ostride + (size_t)j * N + k] = o[j];
  count_exact(fallback, nexact);
}

// Relinearised products in coefficient form and their extension to B: row r = job * 2 + c of
// x = c01 + K (mod Q), K the key sum of the job's unit (jobs_per_unit jobs share one), written to
// xq [rows][L][N] and extended into xb [rows][K][N].
template <int L>
__global__ void __launch_bounds__(TPB) k_add_ext_q_to_b(Tables T, const uint64_t* __restrict__ c01,
                                                       const uint64_t* __restrict__ key, int jobs_per_unit,
                                                       uint64_t* __restrict__ xq, uint64_t* __restrict__ xb,
                                                       uint32_t* fallback) {
  const Consts& C = *T.c;
  constexpr int K = L + 1;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const size_t row = blockIdx.y;
  if (k >= N) return;
  const size_t job = row / 2, comp = row % 2, unit = job / jobs_per_unit;
  uint64_t x[L], o[K];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    x[i] = addmod(c01[(row * L + i) * N + k], key[((unit * 2 + comp) * L + i) * N + k], C.prm[i].p);
    xq[(row * L + i) * N + k] = x[i];
  }
  uint32_t nexact = 0;
  ext_one<L>(C, x, o, nexact);
#pragma unroll
  for (int j = 0; j < K; ++j) xb[(row * K + j) * N + k] = o[j];
  count_exact(fallback, nexact);
}

// alpha[b][r][p]: constant added at every NTT position of c0, limb p, for f_r = S + Delta [-r]_t.
template <int L>
__global__ void k_factor_constants(Tables T, const uint64_t* __restrict__ scoef, int nb, int h,
                                   uint64_t* __restrict__ alpha, uint32_t* fallback) {
  const Consts& C = *T.c;
  constexpr int K = L + 1;
  const int N = C.n;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * h) return;
  const int b = idx / h, r = idx % h;
  uint64_t x[L], xr[L], e0[K], er[K];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint64_t q = C.prm[i].p;
    x[i] = scoef[((size_t)b * 2 * L + i) * N];                     // c0, limb i, coefficient 0
    const uint64_t rd = mulmod(C.delta[i], (uint64_t)r, C.prm[i]);  // r Delta mod q_i
    xr[i] = submod(x[i], rd, q);
  }
  uint32_t nexact = 0;
  ext_one<L>(C, x, e0, nexact);
  ext_one<L>(C, xr, er, nexact);
  uint64_t* out = alpha + (size_t)idx * (L + K);
#pragma unroll
  for (int i = 0; i < L; ++i) out[i] = submod(xr[i], x[i], C.prm[i].p);
#pragma unroll
  for (int j = 0; j < K; ++j) out[L + j] = submod(er[j], e0[j], C.prm[L + j].p);
  count_exact(fallback, nexact);
}

// s = delta_2u + delta_2u+1 mod p and floor(s 2^64 / p) for every (pair, job u, prime p).
__global__ void __launch_bounds__(TPB) k_pair_constants(Tables T, const uint64_t* __restrict__ alpha, int npairs,
                                                       int h, uint64_t* __restrict__ pconst) {
  const Consts& C = *T.c;
  const int P = C.L + C.K, J0 = h / 2;
  const int idx = blockIdx.x * TPB + threadIdx.x;
  if (idx >= npairs * J0 * P) return;
  const int p = idx % P, u = (idx / P) % J0, pair = idx / (P * J0);
  const uint64_t q = C.prm[p].p;
  const uint64_t s = addmod(alpha[((size_t)pair * h + 2 * u) * P + p], alpha[((size_t)pair * h + 2 * u + 1) * P + p], q);
  pconst[2 * (size_t)idx] = s;
  pconst[2 * (size_t)idx + 1] = shoup_companion(s, q);
}

__device__ __forceinline__ void tensor_at(const Consts& C, const TensorJob& J, int k, int p) {
  const int N = C.n, L = C.L, K = C.K, P = L + K;
  const Prime& pr = C.prm[p];
  uint64_t x0, x1, y0, y1;
  if (p < L) {
    x0 = J.xq[(size_t)p * N + k]; x1 = J.xq[(size_t)(L + p) * N + k];
    y0 = J.yq[(size_t)p * N + k]; y1 = J.yq[(size_t)(L + p) * N + k];
  } else {
    x0 = J.xb[(size_t)(p - L) * N + k]; x1 = J.xb[(size_t)(K + p - L) * N + k];
    y0 = J.yb[(size_t)(p - L) * N + k]; y1 = J.yb[(size_t)(K + p - L) * N + k];
  }
  if (J.ax) x0 = addmod(x0, J.ax[p], pr.p);
  if (J.ay) y0 = addmod(y0, J.ay[p], pr.p);
  J.d[(size_t)p * N + k] = mulmod(x0, y0, pr);
  const u128 m = (u128)x0 * y1 + (u128)x1 * y0;
  J.d[(size_t)(P + p) * N + k] = reduce116((uint64_t)m, (uint64_t)(m >> 64), pr);
  J.d[(size_t)(2 * P + p) * N + k] = mulmod(x1, y1, pr);
}

__global__ void __launch_bounds__(TPB) k_tensor(Tables T, const TensorJob* __restrict__ jobs) {
  const Consts& C = *T.c;
  const int k = blockIdx.x * TPB + threadIdx.x;
  if (k >= C.n) return;
  tensor_at(C, jobs[blockIdx.z], k, (int)blockIdx.y);
}

// One tensor job passed by value (no job array in device memory).
__global__ void __launch_bounds__(TPB) k_tensor_one(Tables T, TensorJob J) {
  const Consts& C = *T.c;
  const int k = blockIdx.x * TPB + threadIdx.x;
  if (k >= C.n) return;
  tensor_at(C, J, k, (int)blockIdx.y);
}

// First tree level.  Every factor is f_r = X + delta_r (X the select-and-sum ciphertext, delta_r
// an integer added to coefficient 0 of c0, the exact difference of the centred lifts), so over
// the integers
//   (X + delta_a) (X + delta_b) = (X0^2 + s X0 + p,  2 X0 X1 + s X1,  X1^2),
// s = delta_a + delta_b, p = delta_a delta_b.  The three products of X are formed once per pair
// here; k_scale_round<L, true> adds the linear terms of each job in coefficient form.
__global__ void __launch_bounds__(TPB) k_square(Tables T, const uint64_t* __restrict__ xq,
                                               const uint64_t* __restrict__ xb, uint64_t* __restrict__ d) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L, K = C.K, P = L + K;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int p = blockIdx.y;
  const size_t pair = blockIdx.z;
  if (k >= N) return;
  const Prime& pr = C.prm[p];
  uint64_t x0, x1;
  if (p < L) {
    x0 = xq[((pair * 2 + 0) * L + p) * N + k];
    x1 = xq[((pair * 2 + 1) * L + p) * N + k];
  } else {
    x0 = xb[((pair * 2 + 0) * K + p - L) * N + k];
    x1 = xb[((pair * 2 + 1) * K + p - L) * N + k];
  }
  d[((pair * 3 + 0) * P + p) * N + k] = mulmod(x0, x0, pr);
  d[((pair * 3 + 1) * P + p) * N + k] = mulmod(addmod(x0, x0, pr.p), x1, pr);
  d[((pair * 3 + 2) * P + p) * N + k] = mulmod(x1, x1, pr);
}

// round(t d / Q) into B, then the centred B -> Q extension.  Components 0 and 1 of every job go
// to c01 [job][2][L][N], component 2 to c2 [unit][L][N].
//   FIRST = false: d [job][3][P][N], one unit per job (poly = job * 3 + component).
//   FIRST = true:  d [pair][3][P][N] holds the products of X (k_square); each pair has J0 jobs
//                  (factors 2u, 2u + 1) sharing one component 2, poly = pair * (2 J0 + 1) + e.
template <int L, bool FIRST>
__global__ void __launch_bounds__(TPB) k_scale_round(Tables T, const uint64_t* __restrict__ d,
                                                    const uint64_t* __restrict__ xq,
                                                    const uint64_t* __restrict__ xb,
                                                    const uint64_t* __restrict__ alpha,
                                                    const uint64_t* __restrict__ pconst, int h, int J0,
                                                    uint64_t* __restrict__ c01, uint64_t* __restrict__ c2,
                                                    uint32_t* fallback) {
  const Consts& C = *T.c;
  constexpr int K = L + 1, P = L + K;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const size_t poly = blockIdx.y;
  if (k >= N) return;
  const uint64_t* src;
  uint64_t* dst;
  size_t pair = 0;
  int u = 0, comp;
  bool lin = false;
  if (FIRST) {
    const int per = 2 * J0 + 1, pi = (int)blockIdx.y;   // 32-bit division: far cheaper than 64-bit
    pair = (size_t)(pi / per);
    const int e = pi % per;
    if (e < 2 * J0) {
      u = e >> 1;
      comp = e & 1;
      lin = true;
      src = d + (pair * 3 + comp) * P * N;
      dst = c01 + ((pair * J0 + u) * 2 + comp) * L * N;
    } else {
      comp = 2;
      src = d + (pair * 3 + 2) * P * N;
      dst = c2 + pair * L * N;
    }
  } else {
    const size_t job = poly / 3;
    comp = (int)(poly % 3);
    src = d + poly * P * N;
    dst = comp < 2 ? c01 + (job * 2 + comp) * L * N : c2 + job * L * N;
  }
  // per-limb row bases, formed once (uniform)
  const uint64_t* srck = src + k;
  const uint64_t *xqk = nullptr, *xbk = nullptr, *scb = nullptr, *al = nullptr;
  if (FIRST && lin) {
    xqk = xq + (pair * 2 + comp) * L * N + k;
    xbk = xb + (pair * 2 + comp) * K * N + k;
    scb = pconst + (pair * J0 + u) * P * 2;     // per limb: s = delta_a + delta_b, its companion
    al = alpha + (pair * h + 2 * u) * P;         // delta_a; delta_b follows P words later
  }
  uint64_t y[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    uint64_t v = srck[(size_t)p * N];
    if (FIRST && lin) {
      const Prime& pr = C.prm[p];
      const uint64_t xv = p < L ? xqk[(size_t)p * N] : xbk[(size_t)(p - L) * N];
      v = addmod(v, shoup(xv, scb[2 * p], scb[2 * p + 1], pr.p), pr.p);
      if (comp == 0 && k == 0) v = addmod(v, mulmod(al[p], al[P + p], pr), pr.p);
    }
    y[p] = shoup(v, C.phat_inv[p], C.phat_inv_shoup[p], C.prm[p].p);
  }
  FixAcc a{0, 0};
#pragma unroll
  for (int i = 0; i < L; ++i) fix_add96(a, y[i], C.theta[i]);
  bool amb;
  uint32_t nexact = 0;
  uint64_t R = fix_round96(a, L, &amb);
  if (amb) {
    // frac(sum y_i r_i / q_i) > 1/2  <=>  the integer with residues y_i r_i (Q/q_i) exceeds Q/2
    uint64_t z[L];
#pragma unroll
    for (int i = 0; i < L; ++i) z[i] = mulmod(y[i], C.tb_mod_q[i], C.prm[i]);
    bool gt;
    crt_exact(z, L, C.qhat_w, C.Qw, &gt, nullptr);
    R = a.ip + (gt ? 1 : 0);
    ++nexact;
  }
  // z_j = round(t d / Q) mod b_j
  uint64_t yb[K];
  Split27 yq[L];
#pragma unroll
  for (int i = 0; i < L; ++i) yq[i] = split27(y[i]);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const Prime& pr = C.prm[L + j];
    Acc3 acc;
    acc.mac(split27(y[L + j]), C.tbhat_mod_b[j]);
    acc.add(R);
#pragma unroll
    for (int i = 0; i < L; ++i) acc.mac(yq[i], C.omega_mod_b[i][j]);
    const uint64_t zj = acc.reduce_lazy(pr);
    yb[j] = shoup(zj, C.bhat_inv[j], C.bhat_inv_shoup[j], pr.p);
  }
  uint64_t v = round_fp<K>(yb, C.inv_b_d, &amb);
  if (amb) v = exact_round_b<K>(C, yb, nexact);
  Split27 ybs[K];
#pragma unroll
  for (int j = 0; j < K; ++j) ybs[j] = split27(yb[j]);
  const Split27 vs = split27(v);
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const Prime& pr = C.prm[i];
    Acc3 acc;
    acc.mac(vs, pr.p - C.b_mod_q[i]);
#pragma unroll
    for (int j = 0; j < K; ++j) acc.mac(ybs[j], C.bhat_mod_q[j][i]);
    dst[(size_t)i * N + k] = acc.reduce(pr);
  }
  count_exact(fallback, nexact);
}

// D_i = [c2 (Q/q_i)^-1]_{q_i} of every unit, as residues mod every q_j: D [unit][i][j][N].
template <int L>
__global__ void __launch_bounds__(TPB) k_relin_digits(Tables T, const uint64_t* __restrict__ c2,
                                                     uint64_t* __restrict__ D) {
  const Consts& C = *T.c;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const size_t row = blockIdx.y;
  if (k >= N) return;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint64_t v = c2[(row * L + i) * N + k];
    const uint64_t Di = shoup(v, C.qhat_inv[i], C.qhat_inv_shoup[i], C.prm[i].p);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const uint64_t q = C.prm[j].p;
      D[((row * L + i) * L + j) * N + k] = Di >= q ? Di - q : Di;
    }
  }
}

// out[job] = c01h[job] + sum_i Dhat_i (.) rlk_i for the jobs_per_unit jobs of each unit (they
// share one component 2, so the key sum is formed once).  unit / units_per_pair is the pair
// b * nq + q, whose query q selects the key.
template <int L>
__global__ void __launch_bounds__(TPB) k_relin_inner(Tables T, const uint64_t* __restrict__ c01h,
                                                    const uint64_t* __restrict__ Dhat,
                                                    const uint64_t* __restrict__ rlk_base, long rlk_stride,
                                                    const int* __restrict__ qslot, int jobs_per_unit,
                                                    int units_per_pair, int nq, uint64_t* __restrict__ out) {
  const Consts& C = *T.c;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int j = blockIdx.y;
  // The units of one query follow each other in launch order (when every query has as many), so
  // that its key's rows stay in L2 while they are read; unit = pair * units_per_pair + r with
  // pair = b * nq + q.
  size_t unit = blockIdx.z;
  int q;
  const size_t per_q = gridDim.z / nq;
  if (gridDim.z % ((size_t)nq * units_per_pair) == 0) {
    q = (int)(blockIdx.z / per_q);
    const size_t rz = blockIdx.z % per_q;
    unit = ((rz / units_per_pair) * nq + q) * units_per_pair + rz % units_per_pair;
  } else {
    q = (int)((unit / units_per_pair) % nq);
  }
  if (k >= N) return;
  const Prime& pr = C.prm[j];
  const uint64_t* rlk = rlk_base + (size_t)(qslot ? qslot[q] : q) * rlk_stride;
  u128 a0 = 0, a1 = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const uint64_t dv = Dhat[((unit * L + i) * L + j) * N + k];
    a0 += (u128)dv * rlk[(((size_t)i * 2 + 0) * L + j) * N + k];
    a1 += (u128)dv * rlk[(((size_t)i * 2 + 1) * L + j) * N + k];
  }
  const uint64_t r0 = reduce116((uint64_t)a0, (uint64_t)(a0 >> 64), pr);
  const uint64_t r1 = reduce116((uint64_t)a1, (uint64_t)(a1 >> 64), pr);
  for (int u = 0; u < jobs_per_unit; ++u) {
    const size_t job = unit * jobs_per_unit + u;
    const size_t o0 = ((job * 2 + 0) * L + j) * N + k, o1 = ((job * 2 + 1) * L + j) * N + k;
    out[o0] = c01h ? addmod(r0, c01h[o0], pr.p) : r0;
    out[o1] = c01h ? addmod(r1, c01h[o1], pr.p) : r1;
  }
}

// acc[slot(q)] += sum over batches b of x[b * nq + q]: entries of `rows` rows of N residues,
// row r modulo q_(r mod L), xstride words apart in x and astride words apart in acc.
// Accumulations run a thread per coefficient down the batches: small workgroups (more of them
// in flight) and AU loads issued together per thread keep enough reads outstanding.
constexpr int ATPB = 64, AU = 8;
__global__ void __launch_bounds__(ATPB) k_accumulate(Tables T, const uint64_t* __restrict__ x,
                                                    long xstride, int nb, int nq, const int* __restrict__ qslot,
                                                    uint64_t* __restrict__ acc, long astride) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int k = blockIdx.x * ATPB + threadIdx.x;
  const int cl = blockIdx.y;
  const int q = blockIdx.z;
  if (k >= N) return;
  const Prime& pr = C.prm[cl % L];
  uint64_t* a = acc + (size_t)(qslot ? qslot[q] : q) * astride;
  uint64_t s = a[(size_t)cl * N + k];
  int b = 0;
  while (b < nb) {
    u128 t = s;
    const int end = min(nb, b + 1000);             // 1000 * 2^54 stays below 2^116
    for (; b + AU <= end; b += AU) {
      uint64_t v[AU];
#pragma unroll
      for (int i = 0; i < AU; ++i) v[i] = x[((size_t)(b + i) * nq + q) * xstride + (size_t)cl * N + k];
#pragma unroll
      for (int i = 0; i < AU; ++i) t += v[i];
    }
    for (; b < end; ++b) t += x[((size_t)b * nq + q) * xstride + (size_t)cl * N + k];
    s = reduce116((uint64_t)t, (uint64_t)(t >> 64), pr);
  }
  a[(size_t)cl * N + k] = s;
}

// acc[slot(q)] [i][j] += sum over batches b of the relinearisation digit D_i of c2[b * nq + q],
// taken mod q_j (the digits are formed here, not stored): D_i = [c2_i (Q/q_i)^-1]_{q_i}.
template <int L>
__global__ void __launch_bounds__(ATPB) k_accumulate_digits(Tables T, const uint64_t* __restrict__ c2, long cstride,
                                                           int nb, int nq, const int* __restrict__ qslot,
                                                           uint64_t* __restrict__ acc, long astride) {
  const Consts& C = *T.c;
  const int N = C.n;
  const int k = blockIdx.x * ATPB + threadIdx.x;
  const int ij = blockIdx.y, i = ij / L, j = ij % L;
  const int q = blockIdx.z;
  if (k >= N) return;
  const Prime& pr = C.prm[j];
  const uint64_t qi = C.prm[i].p, w = C.qhat_inv[i], wq = C.qhat_inv_shoup[i], qj = pr.p;
  uint64_t* a = acc + (size_t)(qslot ? qslot[q] : q) * astride;
  uint64_t s = a[(size_t)ij * N + k];
  const uint64_t* src = c2 + (size_t)i * N + k;
  int b = 0;
  while (b < nb) {
    u128 t = s;
    const int end = min(nb, b + 1000);             // 1000 * 2^54 stays below 2^116
    for (; b + AU <= end; b += AU) {
      uint64_t v[AU];
#pragma unroll
      for (int u = 0; u < AU; ++u) v[u] = src[((size_t)(b + u) * nq + q) * cstride];
#pragma unroll
      for (int u = 0; u < AU; ++u) {
        const uint64_t d = shoup(v[u], w, wq, qi);
        t += d >= qj ? d - qj : d;
      }
    }
    for (; b < end; ++b) {
      const uint64_t d = shoup(src[((size_t)b * nq + q) * cstride], w, wq, qi);
      t += d >= qj ? d - qj : d;
    }
    s = reduce116((uint64_t)t, (uint64_t)(t >> 64), pr);
  }
  a[(size_t)ij * N + k] = s;
}

// acc[slot(q)] += sum over batches b of x[b * nq + q] (.) vhat[b]: the server values of each
// batch (NTT form [L][N], one plaintext per batch) times that batch's equality ciphertexts
// (NTT form [2][L][N], xstride words apart), accumulated per query (NTT form).
__global__ void __launch_bounds__(ATPB) k_value_accumulate(Tables T, const uint64_t* __restrict__ x,
                                                          long xstride, const uint64_t* __restrict__ vhat,
                                                          int nb, int nq, const int* __restrict__ qslot,
                                                          uint64_t* __restrict__ acc, long astride) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int k = blockIdx.x * ATPB + threadIdx.x;
  const int cl = blockIdx.y;                       // component * L + limb
  const int q = blockIdx.z;
  if (k >= N) return;
  const int l = cl % L;
  const Prime& pr = C.prm[l];
  uint64_t* a = acc + (size_t)(qslot ? qslot[q] : q) * astride;
  uint64_t s = a[(size_t)cl * N + k];
  int b = 0;
  while (b < nb) {
    u128 t = s;
    const int end = min(nb, b + 200);              // 200 products below 2^108 stay below 2^116
    for (; b + AU <= end; b += AU) {
      uint64_t v[AU], w[AU];
#pragma unroll
      for (int i = 0; i < AU; ++i) {
        v[i] = x[((size_t)(b + i) * nq + q) * xstride + (size_t)cl * N + k];
        w[i] = vhat[((size_t)(b + i) * L + l) * N + k];
      }
#pragma unroll
      for (int i = 0; i < AU; ++i) t += (u128)v[i] * w[i];
    }
    for (; b < end; ++b)
      t += (u128)x[((size_t)b * nq + q) * xstride + (size_t)cl * N + k] * vhat[((size_t)b * L + l) * N + k];
    s = reduce116((uint64_t)t, (uint64_t)(t >> 64), pr);
  }
  a[(size_t)cl * N + k] = s;
}

// Select-and-sum.  Thread = one slot position k of one limb, IB server batches at a time (the
// client ciphertext value is loaded once and used IB times).  A product of two residues below
// 2^54 is formed from 27-bit halves, a = a1 2^27 + a0 and b = b1 2^27 + b0 (the plaintexts are
// stored pre-split: b0 in the low and b1 in the high 32-bit word), with three products
// (Karatsuba) into three 64-bit accumulators
//   lo += a0 b0,  hi += a1 b1,  ms += (a0 + a1)(b0 + b1),
// so that the middle term a0 b1 + a1 b0 is ms - lo - hi, exactly.  Terms are below 2^56, so
// FOLD = 254 terms (plus a restart value below 2^54) fit in 64 bits; every FOLD terms the value
// lo + (ms - lo - hi) 2^27 + hi 2^54 is reduced and restarts both lo and ms (hi restarts at 0).
// Loads of a partial group are clamped to its last batch so that every load is unconditional
// (results of padding lanes are dropped).  A workgroup's slice is one 256-position block of the
// plaintext store, where the IB batches of a group are one contiguous run per code position.
constexpr int IB = 16;
static_assert(TPB == PT_BLOCK, "a select-and-sum slice is one plaintext-store block");
constexpr int FOLD = 254;
__device__ __forceinline__ uint64_t fold3(uint64_t lo, uint64_t ms, uint64_t hi, const Prime& pr) {
  const uint64_t mid = ms - lo - hi;
  const u128 v = (u128)lo + ((u128)mid << 27) + ((u128)hi << 54);
  return reduce128((uint64_t)v, (uint64_t)(v >> 64), pr);
}

// Block numbering: a slice (TPB positions of one limb) has zg = ceil(nb / IB) batch groups that
// read the same client values.  Workgroups go to the 8 XCDs round-robin, so block b runs on XCD
// b & 7; the zg groups of a slice get consecutive numbers on one XCD, are resident together and
// share the client values through that XCD's L2.
__global__ void __launch_bounds__(TPB) k_select_sum(Tables T, const uint64_t* __restrict__ Cn,
                                                   const uint64_t* __restrict__ Pc, int gs, int bfirst, int ell,
                                                   int nb, uint64_t* __restrict__ S, long sstride, int slices, int zg) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int bid = blockIdx.x, local = bid >> 3;
  const int slice = (local / zg) * 8 + (bid & 7);
  if (slice >= slices) return;
  const int kchunks = N / TPB;
  const int k0 = (slice % kchunks) * TPB;
  const uint32_t tid = threadIdx.x;
  const int k = k0 + (int)tid;
  const int l = slice / kchunks;
  const int b0 = (local % zg) * IB;
  const int nbl = min(IB, nb - b0);
  const Prime& pr = C.prm[l];
  constexpr uint64_t M27 = (1ull << 27) - 1;
  uint64_t lo[2][IB], ms[2][IB], hi[2][IB];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < IB; ++b) lo[c][b] = ms[c][b] = hi[c][b] = 0;
  const size_t pstep = (size_t)L * N * gs, cstep = (size_t)2 * L * N;
  // wave-uniform block bases; each lane adds its position (scalar base + 32-bit lane offset)
  const uint64_t* pb[IB];
#pragma unroll
  for (int b = 0; b < IB; ++b) {
    const int bb = bfirst + b0 + min(b, nbl - 1), G = bb / gs, g = bb % gs;
    pb[b] = Pc + ((((size_t)G * ell * L + l) * kchunks + k0 / PT_BLOCK) * gs + g) * PT_BLOCK;
  }
  const uint64_t* cb = Cn + (size_t)l * N + k0;
  int fold = 0;
  for (int j = 0; j < ell; ++j) {
    uint64_t w[IB];
#pragma unroll
    for (int b = 0; b < IB; ++b) w[b] = __builtin_nontemporal_load(pb[b] + j * pstep + tid);
    const uint64_t c0 = cb[j * cstep + tid], c1 = cb[j * cstep + (size_t)L * N + tid];
    const uint32_t a00 = (uint32_t)(c0 & M27), a01 = (uint32_t)(c0 >> 27);
    const uint32_t a10 = (uint32_t)(c1 & M27), a11 = (uint32_t)(c1 >> 27);
    const uint32_t as0 = a00 + a01, as1 = a10 + a11;
#pragma unroll
    for (int b = 0; b < IB; ++b) {
      const uint32_t blo = (uint32_t)w[b], bhi = (uint32_t)(w[b] >> 32), bs = blo + bhi;
      lo[0][b] += (uint64_t)a00 * blo;
      hi[0][b] += (uint64_t)a01 * bhi;
      ms[0][b] += (uint64_t)as0 * bs;
      lo[1][b] += (uint64_t)a10 * blo;
      hi[1][b] += (uint64_t)a11 * bhi;
      ms[1][b] += (uint64_t)as1 * bs;
    }
    if (++fold == FOLD) {
      fold = 0;
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < IB; ++b) {
          lo[c][b] = ms[c][b] = fold3(lo[c][b], ms[c][b], hi[c][b], pr);
          hi[c][b] = 0;
        }
    }
  }
#pragma unroll
  for (int b = 0; b < IB; ++b)
    if (b < nbl)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        S[(size_t)(b0 + b) * sstride + ((size_t)c * L + l) * N + k] = fold3(lo[c][b], ms[c][b], hi[c][b], pr);
}

// Select-and-sum of several queries against one tile of server plaintexts.
// A workgroup of 4 waves owns 64 slot positions (one per lane) of one limb, MQ = 2 queries and
// MB = 16 batches; wave w computes both queries x batches 4 w + {0..3} (16 outputs per lane,
// three accumulators each as in k_select_sum), loading the next code position's values while
// it multiplies the current ones.  The waves of a workgroup read the same client values (L1),
// and blocks are numbered so that all query groups of one (positions, limb, batch group)
// region are dispatched consecutively to the same XCD and share its L2 for the plaintexts; the
// four regions that cover one 256-position block of the plaintext store follow each other there,
// so that the block's contiguous run is read at about the same time.
constexpr int MQ = 2, MB = 16, MBB = 4, MTPB = 64 * (MB / MBB);
constexpr int MRQ = PT_BLOCK / 64;   // regions per plaintext-store block
__global__ void __launch_bounds__(MTPB) k_select_sum_multi(Tables T, const uint64_t* __restrict__ Cq,
                                                          long cq_stride, const int* __restrict__ qslot, int nq,
                                                          const uint64_t* __restrict__ Pc, int gs, int bfirst,
                                                          int ell, int nb, uint64_t* __restrict__ S, int regions,
                                                          int qgroups) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int bid = blockIdx.x, xcd = bid & 7, w8 = bid >> 3;
  const int qg = w8 % qgroups, r8 = w8 / qgroups;
  const int region = ((r8 / MRQ) * 8 + xcd) * MRQ + r8 % MRQ;
  if (region >= regions) return;
  const int kchunks = N / 64;
  const int kc = region % kchunks, l = (region / kchunks) % L, bg = region / (kchunks * L);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kbase = kc * 64, q0 = qg * MQ, b0 = bg * MB + wave * MBB;
  const int nql = min(MQ, nq - q0), nbl = min(MBB, nb - b0);
  if (nbl <= 0) return;
  const Prime& pr = C.prm[l];
  constexpr uint64_t M27 = (1ull << 27) - 1;
  const size_t cjs = (size_t)2 * L * N, pjs = (size_t)L * N * gs;
  const uint64_t* cp[MQ][2];
  const uint64_t* pp[MBB];
#pragma unroll
  for (int a = 0; a < MQ; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
      cp[a][c] = Cq + (size_t)(qslot ? qslot[q0 + min(a, nql - 1)] : q0 + min(a, nql - 1)) * cq_stride +
                 ((size_t)c * L + l) * N + kbase + lane;
#pragma unroll
  for (int b = 0; b < MBB; ++b) {
    const int bb = bfirst + b0 + min(b, nbl - 1), G = bb / gs, g = bb % gs;
    pp[b] = Pc + ((((size_t)G * ell * L + l) * (N / PT_BLOCK) + kbase / PT_BLOCK) * gs + g) * PT_BLOCK +
            kbase % PT_BLOCK + lane;
  }
  uint64_t lo[MQ][2][MBB], ms[MQ][2][MBB], hi[MQ][2][MBB];
#pragma unroll
  for (int a = 0; a < MQ; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < MBB; ++b) lo[a][c][b] = ms[a][c][b] = hi[a][c][b] = 0;
  uint64_t nc[MQ][2], np[MBB];
#pragma unroll
  for (int a = 0; a < MQ; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) nc[a][c] = cp[a][c][0];
#pragma unroll
  for (int b = 0; b < MBB; ++b) np[b] = pp[b][0];
  int fold = 0;
  for (int j = 0; j < ell; ++j) {
    const int jn = min(j + 1, ell - 1);
    uint32_t a0[MQ][2], a1[MQ][2], as[MQ][2];
#pragma unroll
    for (int a = 0; a < MQ; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const uint64_t v = nc[a][c];
        nc[a][c] = cp[a][c][jn * cjs];
        a0[a][c] = (uint32_t)(v & M27);
        a1[a][c] = (uint32_t)(v >> 27);
        as[a][c] = a0[a][c] + a1[a][c];
      }
    uint64_t pv[MBB];
#pragma unroll
    for (int b = 0; b < MBB; ++b) {
      pv[b] = np[b];
      np[b] = pp[b][jn * pjs];
    }
#pragma unroll
    for (int b = 0; b < MBB; ++b) {
      const uint32_t blo = (uint32_t)pv[b], bhi = (uint32_t)(pv[b] >> 32), bs = blo + bhi;
#pragma unroll
      for (int a = 0; a < MQ; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          lo[a][c][b] += (uint64_t)a0[a][c] * blo;
          hi[a][c][b] += (uint64_t)a1[a][c] * bhi;
          ms[a][c][b] += (uint64_t)as[a][c] * bs;
        }
    }
    if (++fold == FOLD) {
      fold = 0;
#pragma unroll
      for (int a = 0; a < MQ; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int b = 0; b < MBB; ++b) {
            lo[a][c][b] = ms[a][c][b] = fold3(lo[a][c][b], ms[a][c][b], hi[a][c][b], pr);
            hi[a][c][b] = 0;
          }
    }
  }
  const int k = kbase + lane;
#pragma unroll
  for (int a = 0; a < MQ; ++a)
#pragma unroll
    for (int b = 0; b < MBB; ++b)
      if (a < nql && b < nbl)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          S[((size_t)(b0 + b) * nq + q0 + a) * 2 * L * N + ((size_t)c * L + l) * N + k] =
              fold3(lo[a][c][b], ms[a][c][b], hi[a][c][b], pr);
}

// Select-and-sum of many queries on the int8 matrix cores.  For one slot position k and prime
// q_l the batched select-and-sum is a matrix product: rows are the 16 batches of a tile, columns
// the (query, part) pairs, and the contraction runs over the ell code positions.  Every residue
// (< 2^54) is written as seven balanced base-256 digits x = sum_i d_i 256^i, d_i in [-128, 127],
// stored as int8 planes with the code positions innermost in blocks of PL_K = 64.  The 49 digit
// products of a block accumulate exactly in int32 (|T_s| <= 7 ell 2^14) into 13 sums T_s, one
// per weight 256^s, and the exact value sum_s T_s 256^s is recovered in four 64-bit groups of
// four weights (|V_g| < 2^53 <= q_l for ell <= PL_MAX_ELL), each brought into [0, 2 q_l) and
// multiplied by 2^(32 g) mod q_l, with one reduction of the 128-bit total.
typedef int v4i __attribute__((ext_vector_type(4)));
// Plaintext planes of one group of 16 batches of a cache store (group size gs = 16), layout
// [l][k][kb][digit][batch][64].  Wave = one (l, k, kb); lane = (batch, 16-position quarter).
__global__ void __launch_bounds__(TPB) k_plaintext_planes(Tables T, const uint64_t* __restrict__ Pc, int gs,
                                                         int G, int ell, int kbs, int8_t* __restrict__ out) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const size_t w = (size_t)blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
  if (w >= (size_t)L * N * kbs) return;
  const int lane = threadIdx.x & 63, b = lane & 15, g4 = lane >> 4;
  const int kb = (int)(w % kbs);
  const size_t lk = w / kbs;
  const int k = (int)(lk % N), l = (int)(lk / N);
  const uint64_t p = C.prm[l].p;
  constexpr uint64_t M27 = (1ull << 27) - 1;
  const size_t jstep = (size_t)L * N * gs;
  const uint64_t* src = Pc + (size_t)G * ell * jstep + (size_t)l * N * gs + (size_t)(k / PT_BLOCK) * gs * PT_BLOCK +
                        (size_t)b * PT_BLOCK + k % PT_BLOCK;
  int8_t o[PL_DG][16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int j = kb * PL_K + g4 * 16 + e;
    uint64_t x = 0;
    if (j < ell) {
      const uint64_t wd = src[(size_t)j * jstep];
      x = (wd & M27) + (((wd >> 32) & M27) << 27);
      x -= x >= p ? p : 0;
    }
    int8_t d[PL_DG];
    balanced_digits(x, d);
#pragma unroll
    for (int v = 0; v < PL_DG; ++v) o[v][e] = d[v];
  }
#pragma unroll
  for (int v = 0; v < PL_DG; ++v)
    __builtin_memcpy(out + ((w * PL_DG + v) * 16 + b) * PL_K + 16 * g4, o[v], 16);
}
// Request planes of one query, layout [l][k][kb][digit][part][64], from its NTT form
// [ell][2][L][N].  Workgroup = one (l, 32 positions, kb): the threads of one half-wave read 8 code
// positions of both parts for its 32 positions (one 256-byte row segment per load) and write
// their digits byte by byte to LDS as [position][digit][part][64]; the workgroup then copies
// each position's 896 contiguous bytes out.  29 KB of LDS per workgroup, so that 5 fit on a CU.
constexpr int RP_POS = 32;                             // positions per workgroup
constexpr int RP_ROW = PL_DG * 2 * PL_K + 16;          // LDS bytes per position (padded)
__global__ void __launch_bounds__(TPB) k_request_planes(Tables T, const uint64_t* __restrict__ ch, int ell, int kbs,
                                                       int8_t* __restrict__ out) {
  __shared__ __align__(16) int8_t sm[RP_POS * RP_ROW];
  constexpr int JH = TPB / RP_POS, JE = PL_K / JH;      // 8 thread groups of 8 code positions
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int kb = (int)(blockIdx.x % kbs);
  const int blk = (int)(blockIdx.x / kbs);            // (l, RP_POS-position block)
  const int k0 = (blk % (N / RP_POS)) * RP_POS, l = blk / (N / RP_POS);
  const int kk = threadIdx.x % RP_POS, jh = threadIdx.x / RP_POS;
  const uint64_t p = C.prm[l].p;
  int8_t* row = sm + kk * RP_ROW + jh * JE;
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int e = 0; e < JE; ++e) {
      const int j = kb * PL_K + jh * JE + e;
      uint64_t x = 0;
      if (j < ell) {
        x = ch[(((size_t)j * 2 + c) * L + l) * N + k0 + kk];
        x -= x >= p ? p : 0;
      }
      int8_t d[PL_DG];
      balanced_digits(x, d);
#pragma unroll
      for (int u = 0; u < PL_DG; ++u) row[(u * 2 + c) * PL_K + e] = d[u];
    }
  __syncthreads();
  constexpr int CH = PL_DG * 2 * PL_K / 16;             // 16-byte chunks per position
  int8_t* dst = out + ((((size_t)l * N + k0) * kbs + kb) * PL_DG * 2) * PL_K;
  const size_t kstride = (size_t)kbs * PL_DG * 2 * PL_K;
  for (int x = threadIdx.x; x < RP_POS * CH; x += TPB) {
    const int pos = x / CH, r = x % CH;
    uint4 v;
    __builtin_memcpy(&v, sm + pos * RP_ROW + r * 16, 16);
    __builtin_memcpy(dst + pos * kstride + r * 16, &v, 16);
  }
}
// The contraction over a tile of up to 16 HT batches (HT consecutive 16-batch groups of planes,
// gbytes apart).  Workgroup = 4 waves on one (l, k): 4 / HT query octets (16 columns each) x
// the HT groups, so that the HT waves of an octet read its request planes once from L2 and
// share them in L1.  The workgroups of one (l, k) are numbered consecutively on one XCD and
// share its plaintext planes through L2.  S entry of (batch b, query q) at (b * nq + q) * 2 L N,
// as in k_select_sum_multi.
template <int HT>
__global__ void __launch_bounds__(TPB) k_select_sum_planes(Tables T, const int8_t* __restrict__ Pp, long gbytes,
                                                          const int8_t* __restrict__ Cp, long cps,
                                                          const int* __restrict__ qslot, int nq, int nb, int kbs,
                                                          uint64_t* __restrict__ S, int oblocks) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int bid = blockIdx.x, local = bid >> 3;
  const int ob = local % oblocks, lk = (local / oblocks) * 8 + (bid & 7);
  const int l = lk / N, k = lk % N;
  const int lane = threadIdx.x & 63, m = lane & 15, g4 = lane >> 4;
  const int wv = threadIdx.x >> 6, half = wv % HT, oct = ob * (TPB / 64 / HT) + wv / HT;
  if (oct * 8 >= nq || 16 * half >= nb) return;
  const int q = oct * 8 + (m >> 1), c = m & 1;
  const bool live = q < nq;
  const int8_t* pa = Pp + half * gbytes + ((size_t)lk * kbs * PL_DG * 16 + m) * PL_K + 16 * g4;
  const int8_t* pb = Cp + (size_t)(live ? (qslot ? qslot[q] : q) : 0) * cps +
                     ((size_t)lk * kbs * PL_DG * 2 + c) * PL_K + 16 * g4;
  v4i acc[2 * PL_DG - 1];
#pragma unroll
  for (int s2 = 0; s2 < 2 * PL_DG - 1; ++s2) acc[s2] = v4i{0, 0, 0, 0};
  for (int kb = 0; kb < kbs; ++kb) {
    v4i a[PL_DG], bb[PL_DG];
#pragma unroll
    for (int v = 0; v < PL_DG; ++v) a[v] = *reinterpret_cast<const v4i*>(pa + ((size_t)kb * PL_DG + v) * 16 * PL_K);
#pragma unroll
    for (int u = 0; u < PL_DG; ++u)
      bb[u] = live ? *reinterpret_cast<const v4i*>(pb + ((size_t)kb * PL_DG + u) * 2 * PL_K) : v4i{0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < PL_DG; ++v)
#pragma unroll
      for (int u = 0; u < PL_DG; ++u)
        acc[u + v] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[v], bb[u], acc[u + v], 0, 0, 0);
  }
  if (!live) return;
  const Prime& pr = C.prm[l];
  uint64_t wgt[4];
  plane_group_weights(pr, wgt);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = 16 * half + 4 * g4 + i;   // output row of this lane
    if (b >= nb) continue;
    int32_t Ts[PL_WEIGHTS];
#pragma unroll
    for (int s2 = 0; s2 < PL_WEIGHTS; ++s2) Ts[s2] = acc[s2][i];
    S[(((size_t)b * nq + q) * 2 + c) * L * N + (size_t)l * N + k] = plane_recombine(Ts, pr, wgt);
  }
}

// The contraction over a run of ngroups consecutive 16-batch groups of planes in one launch, with
// the request planes of the workgroup's query octet for its (l, k) staged once in LDS (kbs x 896
// bytes per query) and reused by every group, so that a query's request planes are read once per
// run instead of once per tile.  Workgroup = RUN_WAVES waves on one (l, k) and one octet; wave w
// takes groups w, w + RUN_WAVES, ...; the next code-position block's plaintext digits are loaded into one of
// two register buffers while the current block's 49 products run from the other.  Column m of the products is query m mod 8 of the octet, part
// m / 8.  In LDS each (part, query) run of kbs x 448 bytes starts at part RUN_CS + query RUN_QS,
// with RUN_QS = 16 (mod 256) and RUN_CS = 8 RUN_QS = 128 (mod 256): the 16-byte reads of the 16
// columns then fall on 16 distinct 16-byte bank slots of every 256 bytes (and the 8 columns of a
// half wave on 8 distinct slots of every 128), so that the reads of a wave spread over the banks.
// The oblocks workgroups of one (l, k) are numbered consecutively on one XCD and share its
// plaintext planes through L2.  Needs kbs <= PL_RUN_KBS.
__host__ __device__ constexpr int run_qs(int kbs) {
  return kbs * PL_DG * PL_K + (((16 - kbs * PL_DG * PL_K) % 256) + 256) % 256;
}
// RUN_WPE = 2 (the occupancy that the LDS allows) keeps the accumulators in ordinary VGPRs; without
// it the compiler moves them to AGPRs and the products' results pass through extra moves.
constexpr int RUN_WAVES = 4, RUN_TPB = 64 * RUN_WAVES, RUN_WPE = 2;
__global__ void __launch_bounds__(RUN_TPB) __attribute__((amdgpu_waves_per_eu(RUN_WPE))) k_select_sum_planes_run(Tables T, const int8_t* __restrict__ Pp, long gbytes,
                                                              int ngroups, const int8_t* __restrict__ Cp, long cps,
                                                              const int* __restrict__ qslot, int nq, int nb, int kbs,
                                                              uint64_t* __restrict__ S, int oblocks) {
  extern __shared__ __align__(16) int8_t sB[];
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int bid = blockIdx.x, local = bid >> 3;
  const int oct = local % oblocks, lk = (local / oblocks) * 8 + (bid & 7);
  const int l = lk / N, k = lk % N;
  const int lane = threadIdx.x & 63, m = lane & 15, g4 = lane >> 4, wv = threadIdx.x >> 6;
  const int QS = run_qs(kbs), CS = 8 * QS;
  // stage the octet's request planes, source [kb][digit][part][64] per query, zeros past the
  // last query
  // (all of a thread's loads in flight together -- at most two 16-byte chunks per query -- so that
  // the staging costs about one memory latency; a missing query reads query 0's planes and stages
  // zeros)
  const int chunks = kbs * PL_DG * 2 * PL_K / 16;       // 16-byte chunks per query
  static_assert(PL_RUN_KBS * PL_DG * 2 * PL_K / 16 <= 2 * RUN_TPB, "two chunks per thread and query");
  int qs[8];
#pragma unroll
  for (int qi = 0; qi < 8; ++qi) {
    const int q = oct * 8 + qi;
    qs[qi] = q < nq ? (qslot ? qslot[q] : q) : 0;
  }
  uint4 v[8][2];
#pragma unroll
  for (int qi = 0; qi < 8; ++qi) {
    const int8_t* src = Cp + (size_t)qs[qi] * cps + (size_t)lk * chunks * 16;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = threadIdx.x + h * RUN_TPB;
      if (r < chunks) __builtin_memcpy(&v[qi][h], src + (size_t)r * 16, 16);
    }
  }
#pragma unroll
  for (int qi = 0; qi < 8; ++qi)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = threadIdx.x + h * RUN_TPB;
      if (r >= chunks) continue;
      const uint4 w = oct * 8 + qi < nq ? v[qi][h] : uint4{0, 0, 0, 0};
      const int quarter = r & 3, part = (r >> 2) & 1, kd = r >> 3;   // kd = kb * PL_DG + digit
      __builtin_memcpy(sB + part * CS + qi * QS + kd * PL_K + quarter * 16, &w, 16);
    }
  __syncthreads();
  const int q = oct * 8 + (m & 7), c = m >> 3;
  const bool live = q < nq;
  const int8_t* bq = sB + c * CS + (m & 7) * QS + 16 * g4;
  const Prime pr = C.prm[l];                        // a copy: the stores to S do not reload it
  uint64_t wgt[4];
  plane_group_weights(pr, wgt);
  for (int g = wv; g < ngroups; g += RUN_WAVES) {
    const int8_t* pa = Pp + (size_t)g * gbytes + ((size_t)lk * kbs * PL_DG * 16 + m) * PL_K + 16 * g4;
    v4i acc[PL_WEIGHTS];
#pragma unroll
    for (int s2 = 0; s2 < PL_WEIGHTS; ++s2) acc[s2] = v4i{0, 0, 0, 0};
    // two digit buffers used in turn: block kb + 1 loads into one while block kb multiplies from
    // the other
    v4i a0[PL_DG], a1[PL_DG];
#pragma unroll
    for (int v = 0; v < PL_DG; ++v) a0[v] = *reinterpret_cast<const v4i*>(pa + (size_t)v * 16 * PL_K);
    auto block = [&](const v4i (&a)[PL_DG], int kb) {
      v4i bb[PL_DG];
#pragma unroll
      for (int u = 0; u < PL_DG; ++u) bb[u] = *reinterpret_cast<const v4i*>(bq + (kb * PL_DG + u) * PL_K);
#pragma unroll
      for (int v = 0; v < PL_DG; ++v)
#pragma unroll
        for (int u = 0; u < PL_DG; ++u)
          acc[u + v] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[v], bb[u], acc[u + v], 0, 0, 0);
    };
    for (int kb = 0; kb < kbs; kb += 2) {
      if (kb + 1 < kbs) {
#pragma unroll
        for (int v = 0; v < PL_DG; ++v)
          a1[v] = *reinterpret_cast<const v4i*>(pa + ((size_t)(kb + 1) * PL_DG + v) * 16 * PL_K);
      }
      block(a0, kb);
      if (kb + 1 < kbs) {
        if (kb + 2 < kbs) {
#pragma unroll
          for (int v = 0; v < PL_DG; ++v)
            a0[v] = *reinterpret_cast<const v4i*>(pa + ((size_t)(kb + 2) * PL_DG + v) * 16 * PL_K);
        }
        block(a1, kb + 1);
      }
    }
    if (!live) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = 16 * g + 4 * g4 + i;     // output row of this lane
      if (b >= nb) continue;
      int32_t Ts[PL_WEIGHTS];
#pragma unroll
      for (int s2 = 0; s2 < PL_WEIGHTS; ++s2) Ts[s2] = acc[s2][i];
      S[(((size_t)b * nq + q) * 2 + c) * L * N + (size_t)l * N + k] = plane_recombine(Ts, pr, wgt);
    }
  }
}

// Seeded uniform polynomials (request compression): a_{j,l}[k] = W mod q_l, W the 16 bytes
// of the ChaCha20 keystream (RFC 8439; key = the seed, nonce = (j, l, 0)) at 16 k, little-
// endian.  Thread = one 64-byte block = 4 coefficients.
__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }
__device__ __forceinline__ void chacha_qr(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d) {
  a += b; d ^= a; d = rotl32(d, 16);
  c += d; b ^= c; b = rotl32(b, 12);
  a += b; d ^= a; d = rotl32(d, 8);
  c += d; b ^= c; b = rotl32(b, 7);
}
__global__ void __launch_bounds__(TPB) k_expand_uniform(Tables T, ChaChaKey key, int first,
                                                       uint64_t* __restrict__ out, long stride) {
  const Consts& C = *T.c;
  const int N = C.n;
  const int blk = blockIdx.x * TPB + threadIdx.x;    // keystream block = coefficients 4 blk ..
  const int l = blockIdx.y;
  const int jj = blockIdx.z;
  if (4 * blk >= N) return;
  uint32_t s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u};
#pragma unroll
  for (int i = 0; i < 8; ++i) s[4 + i] = key.k[i];
  s[12] = (uint32_t)blk;
  s[13] = (uint32_t)(first + jj);
  s[14] = (uint32_t)l;
  s[15] = 0;
  uint32_t x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = s[i];
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    chacha_qr(x[0], x[4], x[8], x[12]);
    chacha_qr(x[1], x[5], x[9], x[13]);
    chacha_qr(x[2], x[6], x[10], x[14]);
    chacha_qr(x[3], x[7], x[11], x[15]);
    chacha_qr(x[0], x[5], x[10], x[15]);
    chacha_qr(x[1], x[6], x[11], x[12]);
    chacha_qr(x[2], x[7], x[8], x[13]);
    chacha_qr(x[3], x[4], x[9], x[14]);
  }
  const Prime& pr = C.prm[l];
  uint64_t* o = out + (size_t)jj * stride + (size_t)l * N + 4 * blk;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint64_t lo = (uint64_t)(x[4 * c] + s[4 * c]) | (uint64_t)(x[4 * c + 1] + s[4 * c + 1]) << 32;
    const uint64_t hi = (uint64_t)(x[4 * c + 2] + s[4 * c + 2]) | (uint64_t)(x[4 * c + 3] + s[4 * c + 3]) << 32;
    o[c] = reduce128(lo, hi, pr);
  }
}

// Modulus switching to q_0 (response compression): out = [round(q_0 X / Q)]_{q_0} for the
// centred lift X of each coefficient.  With Q' = Q / q_0 this is (X - [X]_{Q'}) / Q', and
// [X]_{Q'} mod q_0 follows from the exact CRT over q_1..q_{L-1} (v reductions by Q', then the
// centring) -- no rounding estimate is involved.  ct [2][L][N] -> out [2][N].
template <int L>
__global__ void __launch_bounds__(TPB) k_mod_switch(Tables T, const uint64_t* __restrict__ ct,
                                                   uint64_t* __restrict__ out) {
  const Consts& C = *T.c;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int comp = blockIdx.y;
  if (k >= N) return;
  const Prime& p0 = C.prm[0];
  const uint64_t x0 = ct[((size_t)comp * L) * N + k];
  uint64_t res = x0;
  if (L > 1) {
    uint64_t y[L > 1 ? L - 1 : 1];
    u128 acc = 0;
#pragma unroll
    for (int i = 1; i < L; ++i) {
      const uint64_t xi = ct[((size_t)comp * L + i) * N + k];
      y[i - 1] = mulmod(xi, C.sw_hat_inv[i - 1], C.prm[i]);
      acc += (u128)y[i - 1] * C.sw_hat_mod_q0[i - 1];
    }
    bool gt;
    const int v = crt_exact(y, L - 1, C.sw_hat_w, C.sw_Qw, &gt, nullptr);
    // [X]_{Q'} mod q_0 = sum y_i (Q'/q_i) - (v + gt) Q'   (mod q_0)
    uint64_t r = reduce128((uint64_t)acc, (uint64_t)(acc >> 64), p0);
    const uint64_t sub = mulmod((uint64_t)(v + (gt ? 1 : 0)) % p0.p, C.sw_q_mod_q0, p0);
    r = submod(r, sub, p0.p);
    res = mulmod(submod(x0, r, p0.p), C.sw_qinv_q0, p0);
  }
  out[(size_t)comp * N + k] = res;
}

__global__ void __launch_bounds__(TPB) k_pointwise(Tables T, const uint64_t* __restrict__ a,
                                                  const uint64_t* __restrict__ b, uint64_t* __restrict__ out,
                                                  int nprimes, int bcast) {
  const Consts& C = *T.c;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int p = blockIdx.y;
  const size_t row = blockIdx.z;
  if (k >= N) return;
  const size_t ia = (row * nprimes + p) * N + k;
  const size_t ib = bcast ? (size_t)p * N + k : ia;
  out[ia] = mulmod(a[ia], b[ib], C.prm[p]);
}

__global__ void __launch_bounds__(TPB) k_add_rows(Tables T, const uint64_t* __restrict__ a,
                                                 const uint64_t* __restrict__ b, uint64_t* __restrict__ out,
                                                 int nprimes) {
  const Consts& C = *T.c;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int p = blockIdx.y;
  const size_t row = blockIdx.z;
  if (k >= N) return;
  const size_t i = (row * nprimes + p) * N + k;
  out[i] = addmod(a[i], b[i], C.prm[p].p);
}

struct KQ { uint64_t k[PEPSI_MAXL]; };
__global__ void __launch_bounds__(TPB) k_scale_const(Tables T, uint64_t* __restrict__ ct, KQ kq) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int cl = blockIdx.y;
  if (k >= N) return;
  const int l = cl % L;
  uint64_t& v = ct[(size_t)cl * N + k];
  v = mulmod(v, kq.k[l], C.prm[l]);
}

__device__ __forceinline__ uint64_t lift_t(uint32_t m, uint64_t q) {
  return m <= (PEPSI_T - 1) / 2 ? (uint64_t)m : q - (uint64_t)(PEPSI_T - m);
}

__global__ void __launch_bounds__(TPB) k_add_plain(Tables T, uint64_t* __restrict__ ct,
                                                  const uint32_t* __restrict__ m) {
  const Consts& C = *T.c;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int l = blockIdx.y;
  if (k >= N) return;
  const Prime& pr = C.prm[l];
  const uint64_t dm = mulmod(C.delta[l], lift_t(m[k], pr.p), pr);
  uint64_t& v = ct[(size_t)l * N + k];
  v = addmod(v, dm, pr.p);
}

__global__ void __launch_bounds__(TPB) k_encrypt_finish(Tables T, const uint32_t* __restrict__ m,
                                                       const uint64_t* __restrict__ as,
                                                       const int32_t* __restrict__ e,
                                                       const uint64_t* __restrict__ a,
                                                       uint64_t* __restrict__ ct) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int l = blockIdx.y;
  const size_t idx = blockIdx.z;
  if (k >= N) return;
  const Prime& pr = C.prm[l];
  const uint64_t q = pr.p;
  const uint64_t dm = mulmod(C.delta[l], lift_t(m[idx * N + k], q), pr);
  const int32_t ev = e[idx * N + k];
  const uint64_t eq = ev >= 0 ? (uint64_t)ev : q - (uint64_t)(-(int64_t)ev);
  const uint64_t v = addmod(as[(idx * L + l) * N + k], eq, q);
  ct[((idx * 2 + 0) * L + l) * N + k] = submod(dm, v, q);
  ct[((idx * 2 + 1) * L + l) * N + k] = a[(idx * L + l) * N + k];
}

template <int L>
__global__ void __launch_bounds__(TPB) k_decrypt_round(Tables T, const uint64_t* __restrict__ x,
                                                      uint32_t* __restrict__ m, uint32_t* fallback) {
  const Consts& C = *T.c;
  const int N = C.n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const size_t idx = blockIdx.y;
  if (k >= N) return;
  uint64_t y[L];
  FixAcc a{0, 0};
#pragma unroll
  for (int i = 0; i < L; ++i) {
    y[i] = shoup(x[(idx * L + i) * N + k], C.qhat_inv[i], C.qhat_inv_shoup[i], C.prm[i].p);
    fix_add(a, y[i], C.t_over_q[i]);
  }
  bool amb;
  uint64_t R = fix_round(a, L, &amb);
  if (amb) {
    uint64_t z[L];
#pragma unroll
    for (int i = 0; i < L; ++i) z[i] = mulmod(y[i], C.t_mod_q[i], C.prm[i]);
    bool gt;
    crt_exact(z, L, C.qhat_w, C.Qw, &gt, nullptr);
    R = a.ip + (gt ? 1 : 0);
    if (fallback) atomicAdd(fallback, 1u);
  }
  m[idx * N + k] = (uint32_t)(R % PEPSI_T);
}

__global__ void __launch_bounds__(TPB) k_noise_bits(Tables T, const uint64_t* __restrict__ x,
                                                   uint32_t* out) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const size_t idx = blockIdx.y;
  if (k >= N) return;
  uint64_t z[PEPSI_MAXL];
  for (int i = 0; i < L; ++i) {
    const uint64_t tx = mulmod(x[(idx * L + i) * N + k], C.t_mod_q[i], C.prm[i]);
    z[i] = shoup(tx, C.qhat_inv[i], C.qhat_inv_shoup[i], C.prm[i].p);
  }
  bool gt;
  uint64_t X[PEPSI_MW];
  crt_exact(z, L, C.qhat_w, C.Qw, &gt, X);
  if (gt) {                                        // centred magnitude Q - X
    uint64_t borrow = 0;
    for (int w = 0; w < PEPSI_MW; ++w) {
      const u128 d = (u128)C.Qw.w[w] - X[w] - borrow;
      X[w] = (uint64_t)d;
      borrow = (uint64_t)(d >> 64) & 1;
    }
  }
  uint32_t bits = 0;
  for (int w = PEPSI_MW - 1; w >= 0; --w)
    if (X[w]) { bits = 64 * w + 64 - __clzll(X[w]); break; }
  atomicMax(out, bits);
}

__global__ void __launch_bounds__(TPB) k_keygen_finish(Tables T, const uint64_t* __restrict__ s2,
                                                      const uint64_t* __restrict__ as,
                                                      const int32_t* __restrict__ e,
                                                      const uint64_t* __restrict__ a,
                                                      uint64_t* __restrict__ rlk) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int l = blockIdx.y;
  const int i = blockIdx.z;
  if (k >= N) return;
  const Prime& pr = C.prm[l];
  const uint64_t q = pr.p;
  const uint64_t g = (l == i) ? mulmod(C.qhat_mod_q[i], s2[(size_t)l * N + k], pr) : 0;
  const int32_t ev = e[(size_t)i * N + k];
  const uint64_t eq = ev >= 0 ? (uint64_t)ev : q - (uint64_t)(-(int64_t)ev);
  const uint64_t v = addmod(as[((size_t)i * L + l) * N + k], eq, q);
  rlk[(((size_t)i * 2 + 0) * L + l) * N + k] = submod(g, v, q);
  rlk[(((size_t)i * 2 + 1) * L + l) * N + k] = a[((size_t)i * L + l) * N + k];
}

// x = c0 + c1 s in NTT form: cth [count][2][L][N], sh [L][N] -> x [count][L][N]
__global__ void __launch_bounds__(TPB) k_phase(Tables T, const uint64_t* __restrict__ cth,
                                              const uint64_t* __restrict__ sh, uint64_t* __restrict__ x) {
  const Consts& C = *T.c;
  const int N = C.n, L = C.L;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int l = blockIdx.y;
  const size_t idx = blockIdx.z;
  if (k >= N) return;
  const Prime& pr = C.prm[l];
  const uint64_t c0 = cth[((idx * 2 + 0) * L + l) * N + k];
  const uint64_t c1 = cth[((idx * 2 + 1) * L + l) * N + k];
  x[(idx * L + l) * N + k] = addmod(c0, mulmod(c1, sh[(size_t)l * N + k], pr), pr.p);
}

// Plain fills and copies as kernels (not memset / memcpy nodes), so that a captured launch
// sequence holds kernels only.
__global__ void __launch_bounds__(TPB) k_fill_words(uint64_t* __restrict__ p, size_t words, uint64_t v) {
  for (size_t i = (size_t)blockIdx.x * TPB + threadIdx.x; i < words; i += (size_t)gridDim.x * TPB) p[i] = v;
}
__global__ void __launch_bounds__(TPB) k_copy_words(uint64_t* __restrict__ dst, const uint64_t* __restrict__ src,
                                                   size_t words) {
  for (size_t i = (size_t)blockIdx.x * TPB + threadIdx.x; i < words; i += (size_t)gridDim.x * TPB) dst[i] = src[i];
}

inline dim3 grid_for(int N, int y, int z = 1) { return dim3((N + TPB - 1) / TPB, y, z); }

#define PEPSI_L_LAUNCH(KERNEL, L, GRID, BLOCK, STREAM, ...)                                  \
  switch (L) {                                                                               \
    case 1: hipLaunchKernelGGL(KERNEL<1>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;       \
    case 2: hipLaunchKernelGGL(KERNEL<2>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;       \
    case 3: hipLaunchKernelGGL(KERNEL<3>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;       \
    case 4: hipLaunchKernelGGL(KERNEL<4>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;       \
    case 5: hipLaunchKernelGGL(KERNEL<5>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;       \
    case 6: hipLaunchKernelGGL(KERNEL<6>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;       \
    case 7: hipLaunchKernelGGL(KERNEL<7>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;       \
    case 8: hipLaunchKernelGGL(KERNEL<8>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break;       \
  }

}  // namespace

void ext_q_to_b(const Tables& T, const Consts& hc, const uint64_t* in, uint64_t* out, long ostride,
                int rows, uint32_t* fb, hipStream_t s) {
  if (rows <= 0) return;
  PEPSI_L_LAUNCH(k_ext_q_to_b, hc.L, grid_for(hc.n, rows), dim3(TPB), s, T, in, out, ostride, fb);
}
void add_ext_q_to_b(const Tables& T, const Consts& hc, const uint64_t* c01, const uint64_t* key, int jobs_per_unit,
                    uint64_t* xq, uint64_t* xb, int rows, uint32_t* fb, hipStream_t s) {
  if (rows <= 0) return;
  PEPSI_L_LAUNCH(k_add_ext_q_to_b, hc.L, grid_for(hc.n, rows), dim3(TPB), s, T, c01, key, jobs_per_unit, xq, xb, fb);
}
void factor_constants(const Tables& T, const Consts& hc, const uint64_t* scoef, int nb, int h,
                      uint64_t* alpha, uint64_t* pconst, uint32_t* fb, hipStream_t s) {
  const int n = nb * h;
  if (n <= 0) return;
  PEPSI_L_LAUNCH(k_factor_constants, hc.L, dim3((n + 63) / 64), dim3(64), s, T, scoef, nb, h, alpha, fb);
  const int np = nb * (h / 2) * (hc.L + hc.K);
  if (np > 0) hipLaunchKernelGGL(k_pair_constants, dim3((np + TPB - 1) / TPB), dim3(TPB), 0, s, T, alpha, nb, h, pconst);
}
void tensor(const Tables& T, const Consts& hc, const TensorJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_tensor, grid_for(hc.n, hc.L + hc.K, njobs), dim3(TPB), 0, s, T, jobs);
}
void tensor_one(const Tables& T, const Consts& hc, const TensorJob& job, hipStream_t s) {
  hipLaunchKernelGGL(k_tensor_one, grid_for(hc.n, hc.L + hc.K), dim3(TPB), 0, s, T, job);
}
void square_products(const Tables& T, const Consts& hc, const uint64_t* xq, const uint64_t* xb, uint64_t* d,
                     int pairs, hipStream_t s) {
  if (pairs <= 0) return;
  hipLaunchKernelGGL(k_square, grid_for(hc.n, hc.L + hc.K, pairs), dim3(TPB), 0, s, T, xq, xb, d);
}
void scale_round(const Tables& T, const Consts& hc, const uint64_t* d, uint64_t* c01, uint64_t* c2, int jobs,
                 uint32_t* fb, hipStream_t s) {
  if (jobs <= 0) return;
  switch (hc.L) {
#define PEPSI_SR(LL) case LL: hipLaunchKernelGGL((k_scale_round<LL, false>), grid_for(hc.n, jobs * 3), dim3(TPB), \
                                                 0, s, T, d, nullptr, nullptr, nullptr, nullptr, 0, 0, c01, c2, fb); \
    break;
    PEPSI_SR(1) PEPSI_SR(2) PEPSI_SR(3) PEPSI_SR(4) PEPSI_SR(5) PEPSI_SR(6) PEPSI_SR(7) PEPSI_SR(8)
#undef PEPSI_SR
  }
}
void scale_round_first(const Tables& T, const Consts& hc, const uint64_t* d, const uint64_t* xq,
                       const uint64_t* xb, const uint64_t* alpha, const uint64_t* pconst, int h, int pairs,
                       uint64_t* c01, uint64_t* c2, uint32_t* fb, hipStream_t s) {
  if (pairs <= 0 || h < 2) return;
  const int J0 = h / 2;
  switch (hc.L) {
#define PEPSI_SR(LL) case LL: hipLaunchKernelGGL((k_scale_round<LL, true>), grid_for(hc.n, pairs * (2 * J0 + 1)), \
                                                 dim3(TPB), 0, s, T, d, xq, xb, alpha, pconst, h, J0, c01, c2, fb); \
    break;
    PEPSI_SR(1) PEPSI_SR(2) PEPSI_SR(3) PEPSI_SR(4) PEPSI_SR(5) PEPSI_SR(6) PEPSI_SR(7) PEPSI_SR(8)
#undef PEPSI_SR
  }
}
void relin_digits(const Tables& T, const Consts& hc, const uint64_t* c2, uint64_t* D, int units,
                  hipStream_t s) {
  if (units <= 0) return;
  PEPSI_L_LAUNCH(k_relin_digits, hc.L, grid_for(hc.n, units), dim3(TPB), s, T, c2, D);
}
void relin_inner(const Tables& T, const Consts& hc, const uint64_t* c01h, const uint64_t* Dhat,
                 const uint64_t* rlk, long rlk_stride, const int* qslot, int jobs_per_unit, int units_per_pair,
                 int nq, uint64_t* out, int units, hipStream_t s) {
  if (units <= 0 || nq <= 0 || units_per_pair <= 0 || jobs_per_unit <= 0) return;   // the kernel divides by them
  PEPSI_L_LAUNCH(k_relin_inner, hc.L, grid_for(hc.n, hc.L, units), dim3(TPB), s, T, c01h, Dhat, rlk,
                 rlk_stride, qslot, jobs_per_unit, units_per_pair, nq, out);
}
void accumulate(const Tables& T, const Consts& hc, const uint64_t* x, long xstride, int nb, int nq,
                int rows, const int* qslot, uint64_t* acc, long astride, hipStream_t s) {
  if (nb <= 0 || nq <= 0 || rows <= 0) return;
  hipLaunchKernelGGL(k_accumulate, dim3((hc.n + ATPB - 1) / ATPB, rows, nq), dim3(ATPB), 0, s, T, x, xstride, nb,
                     nq, qslot, acc, astride);
}
void accumulate_digits(const Tables& T, const Consts& hc, const uint64_t* c2, long cstride, int nb, int nq,
                       const int* qslot, uint64_t* acc, long astride, hipStream_t s) {
  if (nb <= 0 || nq <= 0) return;
  PEPSI_L_LAUNCH(k_accumulate_digits, hc.L, dim3((hc.n + ATPB - 1) / ATPB, hc.L * hc.L, nq), dim3(ATPB), s, T, c2,
                 cstride, nb, nq, qslot, acc, astride);
}
void value_accumulate(const Tables& T, const Consts& hc, const uint64_t* x, long xstride, const uint64_t* vhat,
                      int nb, int nq, const int* qslot, uint64_t* acc, long astride, hipStream_t s) {
  if (nb <= 0 || nq <= 0) return;
  hipLaunchKernelGGL(k_value_accumulate, dim3((hc.n + ATPB - 1) / ATPB, 2 * hc.L, nq), dim3(ATPB), 0, s, T, x,
                     xstride, vhat, nb, nq, qslot, acc, astride);
}
void expand_uniform(const Tables& T, const Consts& hc, const ChaChaKey& key, int first, int count,
                    uint64_t* out, long stride, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_expand_uniform, grid_for(hc.n / 4, hc.L, count), dim3(TPB), 0, s, T, key, first, out,
                     stride);
}
void mod_switch(const Tables& T, const Consts& hc, const uint64_t* ct, uint64_t* out, hipStream_t s) {
  PEPSI_L_LAUNCH(k_mod_switch, hc.L, grid_for(hc.n, 2), dim3(TPB), s, T, ct, out);
}
void select_sum(const Tables& T, const Consts& hc, const uint64_t* Cn, const uint64_t* P, int gs, int bfirst,
                int ell, int nb, uint64_t* S, long sstride, hipStream_t s) {
  if (nb <= 0) return;
  const int slices = hc.n / TPB * hc.L, zg = (nb + IB - 1) / IB;
  hipLaunchKernelGGL(k_select_sum, dim3((slices + 7) / 8 * 8 * zg), dim3(TPB), 0, s, T, Cn, P, gs, bfirst, ell,
                     nb, S, sstride, slices, zg);
}
void select_sum_multi(const Tables& T, const Consts& hc, const uint64_t* Cq, long cq_stride, const int* qslot,
                      int nq, const uint64_t* P, int gs, int bfirst, int ell, int nb, uint64_t* S,
                      hipStream_t s) {
  if (nb <= 0 || nq <= 0) return;
  const int regions = (hc.n / 64) * hc.L * ((nb + MB - 1) / MB);
  const int qgroups = (nq + MQ - 1) / MQ;
  const int blocks = ((regions + 8 * MRQ - 1) / (8 * MRQ)) * 8 * MRQ * qgroups;
  hipLaunchKernelGGL(k_select_sum_multi, dim3(blocks), dim3(MTPB), 0, s, T, Cq, cq_stride, qslot, nq, P, gs,
                     bfirst, ell, nb, S, regions, qgroups);
}
size_t plaintext_plane_group_bytes(const Consts& hc, int ell) {
  return (size_t)hc.L * hc.n * plane_kblocks(ell) * PL_DG * 16 * PL_K;
}
size_t request_plane_bytes(const Consts& hc, int ell) {
  return (size_t)hc.L * hc.n * plane_kblocks(ell) * PL_DG * 2 * PL_K;
}
void plaintext_planes(const Tables& T, const Consts& hc, const uint64_t* P, int gs, int G, int ell, int8_t* out,
                      hipStream_t s) {
  const int kbs = plane_kblocks(ell);
  const size_t waves = (size_t)hc.L * hc.n * kbs;
  hipLaunchKernelGGL(k_plaintext_planes, dim3((unsigned)((waves + TPB / 64 - 1) / (TPB / 64))), dim3(TPB), 0, s, T, P,
                     gs, G, ell, kbs, out);
}
void request_planes(const Tables& T, const Consts& hc, const uint64_t* ch, int ell, int8_t* out, hipStream_t s) {
  const int kbs = plane_kblocks(ell);
  hipLaunchKernelGGL(k_request_planes, dim3((unsigned)((size_t)hc.L * (hc.n / RP_POS) * kbs)), dim3(TPB), 0, s, T,
                     ch, ell, kbs, out);
}
void select_sum_planes(const Tables& T, const Consts& hc, const int8_t* Pp, const int8_t* Cp, long cps,
                       const int* qslot, int nq, int nb, int ell, uint64_t* S, hipStream_t s) {
  if (nb <= 0 || nq <= 0 || nb > 4 * PT_GROUP) return;
  const int ht = nb > 2 * PT_GROUP ? 4 : nb > PT_GROUP ? 2 : 1;
  const int octets = (nq + 7) / 8, per = TPB / 64 / ht, oblocks = (octets + per - 1) / per;
  const int lks = hc.L * hc.n;   // a multiple of 8
  const long gb = (long)plaintext_plane_group_bytes(hc, ell);
  const int kbs = plane_kblocks(ell);
  if (ht == 4)
    hipLaunchKernelGGL(k_select_sum_planes<4>, dim3(lks * oblocks), dim3(TPB), 0, s, T, Pp, gb, Cp, cps, qslot, nq,
                       nb, kbs, S, oblocks);
  else if (ht == 2)
    hipLaunchKernelGGL(k_select_sum_planes<2>, dim3(lks * oblocks), dim3(TPB), 0, s, T, Pp, gb, Cp, cps, qslot, nq,
                       nb, kbs, S, oblocks);
  else
    hipLaunchKernelGGL(k_select_sum_planes<1>, dim3(lks * oblocks), dim3(TPB), 0, s, T, Pp, gb, Cp, cps, qslot, nq,
                       nb, kbs, S, oblocks);
}
void zero_words(uint64_t* p, size_t words, hipStream_t s) {
  if (!words) return;
  const size_t blocks = std::min<size_t>((words + TPB - 1) / TPB, 4096);
  hipLaunchKernelGGL(k_fill_words, dim3((unsigned)blocks), dim3(TPB), 0, s, p, words, (uint64_t)0);
}
void copy_words(uint64_t* dst, const uint64_t* src, size_t words, hipStream_t s) {
  if (!words) return;
  const size_t blocks = std::min<size_t>((words + TPB - 1) / TPB, 4096);
  hipLaunchKernelGGL(k_copy_words, dim3((unsigned)blocks), dim3(TPB), 0, s, dst, src, words);
}
void select_sum_planes_run(const Tables& T, const Consts& hc, const int8_t* Pp, int ngroups, const int8_t* Cp,
                           long cps, const int* qslot, int nq, int nb, int ell, uint64_t* S, hipStream_t s) {
  const int kbs = plane_kblocks(ell);
  if (nb <= 0 || nq <= 0 || ngroups <= 0 || kbs > PL_RUN_KBS) return;
  const int oblocks = (nq + 7) / 8;
  const int lks = hc.L * hc.n;   // a multiple of 8
  const long gb = (long)plaintext_plane_group_bytes(hc, ell);
  const size_t lds = (size_t)2 * 8 * run_qs(kbs);
  hipLaunchKernelGGL(k_select_sum_planes_run, dim3(lks * oblocks), dim3(RUN_TPB), lds, s, T, Pp, gb, ngroups, Cp, cps,
                     qslot, nq, nb, kbs, S, oblocks);
}
void pointwise_mul(const Tables& T, const Consts& hc, const uint64_t* a, const uint64_t* b,
                   uint64_t* out, int rows, int nprimes, bool bcast, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_pointwise, grid_for(hc.n, nprimes, rows), dim3(TPB), 0, s, T, a, b, out,
                     nprimes, bcast ? 1 : 0);
}
void add_rows(const Tables& T, const Consts& hc, const uint64_t* a, const uint64_t* b, uint64_t* out,
              int rows, int nprimes, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_add_rows, grid_for(hc.n, nprimes, rows), dim3(TPB), 0, s, T, a, b, out, nprimes);
}
void scale_const(const Tables& T, const Consts& hc, uint64_t* ct, const uint64_t* kq, hipStream_t s) {
  KQ k;
  for (int l = 0; l < PEPSI_MAXL; ++l) k.k[l] = l < hc.L ? kq[l] : 0;
  hipLaunchKernelGGL(k_scale_const, grid_for(hc.n, 2 * hc.L), dim3(TPB), 0, s, T, ct, k);
}
void add_plain_poly(const Tables& T, const Consts& hc, uint64_t* ct, const uint32_t* m, hipStream_t s) {
  hipLaunchKernelGGL(k_add_plain, grid_for(hc.n, hc.L), dim3(TPB), 0, s, T, ct, m);
}
void encrypt_finish(const Tables& T, const Consts& hc, const uint32_t* m, const uint64_t* as,
                    const int32_t* e, const uint64_t* a, uint64_t* ct, int count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_encrypt_finish, grid_for(hc.n, hc.L, count), dim3(TPB), 0, s, T, m, as, e, a, ct);
}
void decrypt_round(const Tables& T, const Consts& hc, const uint64_t* x, uint32_t* m, int count,
                   uint32_t* fb, hipStream_t s) {
  if (count <= 0) return;
  PEPSI_L_LAUNCH(k_decrypt_round, hc.L, grid_for(hc.n, count), dim3(TPB), s, T, x, m, fb);
}
void noise_bits(const Tables& T, const Consts& hc, const uint64_t* x, int count, uint32_t* out,
                hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_noise_bits, grid_for(hc.n, count), dim3(TPB), 0, s, T, x, out);
}
void phase_ntt(const Tables& T, const Consts& hc, const uint64_t* cth, const uint64_t* sh, uint64_t* x,
               int count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_phase, grid_for(hc.n, hc.L, count), dim3(TPB), 0, s, T, cth, sh, x);
}
void keygen_finish(const Tables& T, const Consts& hc, const uint64_t* s2, const uint64_t* as,
                   const int32_t* e, const uint64_t* a, uint64_t* rlk, hipStream_t s) {
  hipLaunchKernelGGL(k_keygen_finish, grid_for(hc.n, hc.L, hc.L), dim3(TPB), 0, s, T, s2, as, e, a, rlk);
}

}  // namespace pepsi
