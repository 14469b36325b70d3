// Kernel launchers (all asynchronous on the given stream).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "params.hpp"
#include "planes.hpp"

namespace pepsi {

// ---------------- negacyclic NTT over the RNS primes ----------------
// Row r of a [rows][N] array is transformed modulo prime (first + r % nprimes).
// Forward: coefficient order in, bit-reversed evaluation order out:
//   out[k] = a(psi^(2 brv(k) + 1)).   Inverse: the exact inverse.
enum NttLoad { LOAD_U64 = 0, LOAD_LIFT_T = 1, LOAD_I8 = 2, LOAD_I32 = 3, LOAD_DIGITS = 4 };
enum NttStore { STORE_U64 = 0, STORE_PLAINTEXT = 1 };

// Server plaintexts in NTT form (STORE_PLAINTEXT).  Each residue is split into 27-bit halves (low
// half in the low, high half in the high 32-bit word).  A store holds groups of gs batches; within
// a group the batches are interleaved per block of 256 positions: the word of batch b = G gs + g,
// code position j, limb l and position k is at
//   ((((G ell + j) L + l) (N / 256) + k / 256) gs + g) 256 + k % 256,
// so that one block of a group's batches is one contiguous run, and a group is one contiguous
// region (space for whole groups is allocated).  A launch over rows (i ell + j) L + l writes
// batch bbase + i.
constexpr int PT_BLOCK = 256, PT_GROUP = 16;
struct PtLayout { int ell = 0, gs = 0, bbase = 0; };

// in: LOAD_U64 -> const uint64_t[rows][N]; LOAD_LIFT_T -> const uint32_t[rows / nprimes][N]
// (a plaintext mod t, lifted to its centred representative); LOAD_I8 / LOAD_I32 -> small
// signed integers [rows / nprimes][N]; LOAD_DIGITS -> the relinearisation digits of component-2
// rows c2 [units][L][N] (coefficient form), formed while loading: row r of [units][L][L] (with
// nprimes = L) is D_i = [c2_i (Q/q_i)^-1]_{q_i} taken mod q_j, i = (r / L) % L, j = r % L.
void ntt_forward(const Tables& T, int logn, const void* in, NttLoad load, void* out,
                 NttStore store, int rows, int nprimes, int first, hipStream_t s);
// Plaintext rows mod t ([nb][ell][N] u32) lifted, transformed over q_0..q_{L-1} and stored into a
// plaintext store of groups of pl.gs batches as batches pl.bbase .. pl.bbase + nb - 1.
void ntt_forward_plaintexts(const Tables& T, int logn, const uint32_t* in, uint64_t* out, int nb, int L,
                            const PtLayout& pl, hipStream_t s);
void ntt_inverse(const Tables& T, int logn, const uint64_t* in, uint64_t* out, int rows,
                 int nprimes, int first, hipStream_t s);
// Inverse transforms of ciphertext products over Q u B formed while loading (P = L + K primes,
// rows [units][3][P] into out [units][3][P][N]):
//   INV_SQUARES: unit = pair, the products (X0^2, 2 X0 X1, X1^2) of X given in NTT form as
//                xq [pairs][2][L][N] and xb [pairs][2][K][N];
//   INV_TENSOR:  unit = job, the tensor (x0 y0, x0 y1 + x1 y0, x1 y1) of TensorJob jobs[job]
//                (with its constants added to c0).
struct TensorJob;
enum InvProducts { INV_SQUARES = 1, INV_TENSOR = 2 };
void ntt_inverse_products(const Tables& T, int logn, InvProducts mode, const uint64_t* xq, const uint64_t* xb,
                          const TensorJob* jobs, uint64_t* out, int units, int nprimes, hipStream_t s);

// ---------------- batching over Z_t ----------------
// slots (natural order, slot k <-> psi_t^(2k+1)) -> plaintext polynomial, coefficients in [0, t)
void encode_slots(const Tables& T, int logn, const uint32_t* slots, uint32_t* poly, int rows,
                  hipStream_t s);
// plaintext polynomial -> slots
void decode_slots(const Tables& T, int logn, const uint32_t* poly, uint32_t* slots, int rows,
                  hipStream_t s);
// server plaintexts of batches [b0, b0 + nb): row (b, j) has slot k = [j in cw[b][k][0..h)]
void encode_server_planes(const Tables& T, int logn, const uint16_t* cw, int h, int ell, int b0,
                          int nb, uint32_t* poly, hipStream_t s);

// ---------------- RNS kernels ----------------
// Q -> B extension of the centred lift: in [rows][L][N] (coefficients mod q), out [rows][K][N]
// (out row stride ostride words between consecutive input rows, starting at limb 0 of B).
void ext_q_to_b(const Tables& T, const Consts& hc, const uint64_t* in, uint64_t* out,
                long ostride, int rows, uint32_t* fallback_count, hipStream_t s);
// x = c01 + key (mod Q) for rows r = job * 2 + c (c01 [jobs][2][L][N], key [units][2][L][N] with
// jobs_per_unit jobs per unit, both coefficient form) into xq [rows][L][N], and its centred Q -> B
// extension into xb [rows][K][N].
void add_ext_q_to_b(const Tables& T, const Consts& hc, const uint64_t* c01, const uint64_t* key, int jobs_per_unit,
                    uint64_t* xq, uint64_t* xb, int rows, uint32_t* fallback_count, hipStream_t s);
// The h factor constants of one select-and-sum ciphertext per batch: alpha[b][r][p] is
// added to every NTT position of c0's limb p for f_r = S + Delta * [-r]_t.
// scoef: coefficient form [nb][2][L][N] (only coefficient 0 of c0 is read).
// Also, for every pair and first-level job u (factors 2u, 2u + 1), the sum s = delta_2u +
// delta_2u+1 mod every prime of Q u B and its Shoup companion: pconst [nb][h / 2][L + K][2].
void factor_constants(const Tables& T, const Consts& hc, const uint64_t* scoef, int nb, int h,
                      uint64_t* alpha, uint64_t* pconst, uint32_t* fallback_count, hipStream_t s);
// Tensor of two extended ciphertexts in NTT form, each given as its Q part [2][L][N] and
// its B part [2][K][N], with optional constants (per limb of Q u B, may be null) added to
// every position of c0: d = [3][L+K][N] (limb p of Q u B at row p).
struct TensorJob {
  const uint64_t* xq; const uint64_t* xb; const uint64_t* yq; const uint64_t* yb;
  const uint64_t* ax; const uint64_t* ay; uint64_t* d;
};
void tensor(const Tables& T, const Consts& hc, const TensorJob* jobs_dev, int njobs, hipStream_t s);
// the same for one job given by value
void tensor_one(const Tables& T, const Consts& hc, const TensorJob& job, hipStream_t s);
// First tree level: d[p] = (X0^2, 2 X0 X1, X1^2) over Q u B for each pair's select-and-sum X,
// given in NTT form as xq [pairs][2][L][N] and xb [pairs][2][K][N]; d [pairs][3][L+K][N].
void square_products(const Tables& T, const Consts& hc, const uint64_t* xq, const uint64_t* xb, uint64_t* d,
                     int pairs, hipStream_t s);
// round(t d / Q) for d over Q u B (coefficient form [jobs][3][L+K][N]), mod Q: components 0, 1
// to c01 [jobs][2][L][N], component 2 to c2 [jobs][L][N].
void scale_round(const Tables& T, const Consts& hc, const uint64_t* d, uint64_t* c01, uint64_t* c2, int jobs,
                 uint32_t* fallback_count, hipStream_t s);
// The same for the h / 2 first-level products (f_2u, f_2u+1) of each pair, f_r = X + delta_r:
// d = square_products output after the inverse NTT; xq, xb: X in coefficient form over Q and B;
// alpha [pairs][h][L+K] = delta_r mod each prime.  c01 [pairs * h/2][2][L][N], c2 [pairs][L][N]
// (component 2 is X1^2 for every product of a pair).
void scale_round_first(const Tables& T, const Consts& hc, const uint64_t* d, const uint64_t* xq,
                       const uint64_t* xb, const uint64_t* alpha, const uint64_t* pconst, int h, int pairs,
                       uint64_t* c01, uint64_t* c2, uint32_t* fallback_count, hipStream_t s);
// relinearisation digits: c2 [units][L][N] coefficient form -> D [units][L][L][N]
void relin_digits(const Tables& T, const Consts& hc, const uint64_t* c2, uint64_t* D, int units,
                  hipStream_t s);
// out[job][c] = c01h[job][c] + sum_i Dhat[unit]_i * rlk_i,c (all NTT form) for the jobs_per_unit
// jobs of each unit (job = unit * jobs_per_unit + u), or the key sum alone when c01h is null;
// c01h, out [jobs][2][L][N], Dhat
// [units][L][L][N].  Unit u belongs to pair u / units_per_pair, pair = b * nq + q, and uses the
// key rlk + slot(q) * rlk_stride ([L][2][L][N] each), where slot(q) = qslot[q] (device array) or
// q when qslot is null; likewise for the other per-query arrays below.
void relin_inner(const Tables& T, const Consts& hc, const uint64_t* c01h, const uint64_t* Dhat,
                 const uint64_t* rlk, long rlk_stride, const int* qslot, int jobs_per_unit, int units_per_pair,
                 int nq, uint64_t* out, int units, hipStream_t s);
// acc[slot(q)] += sum over b < nb of x[b * nq + q]; entries are `rows` rows of N residues (row r
// modulo q_(r mod L)), xstride words apart in x and astride words apart in acc.
void accumulate(const Tables& T, const Consts& hc, const uint64_t* x, long xstride, int nb, int nq,
                int rows, const int* qslot, uint64_t* acc, long astride, hipStream_t s);
// acc[slot(q)][2][L][N] += sum over b < nb of x[b * nq + q] (.) vhat[b] (NTT form; vhat
// [nb][L][N], the server-value plaintexts of the batches; x entries xstride words apart).
void value_accumulate(const Tables& T, const Consts& hc, const uint64_t* x, long xstride, const uint64_t* vhat,
                      int nb, int nq, const int* qslot, uint64_t* acc, long astride, hipStream_t s);
// Request compression: out[j * stride + l * N + k] = a_{first + j, l}[k] for j < count, the
// uniform polynomials expanded from a 32-byte seed with ChaCha20 (key words little-endian).
struct ChaChaKey { uint32_t k[8]; };
void expand_uniform(const Tables& T, const Consts& hc, const ChaChaKey& key, int first, int count,
                    uint64_t* out, long stride, hipStream_t s);
// Response compression: out [2][N] = [round(q_0 X / Q)]_{q_0} of every coefficient X of ct [2][L][N].
void mod_switch(const Tables& T, const Consts& hc, const uint64_t* ct, uint64_t* out, hipStream_t s);
// select-and-sum: S[b][c][l][k] = sum_j C[j][c][l][k] * P[b][j][l][k] mod q_l.
// C: NTT form [ell][2][L][N]; P: a plaintext store of groups of gs batches, of which batches
// bfirst .. bfirst + nb - 1 are summed; S rows of stride sstride.
void select_sum(const Tables& T, const Consts& hc, const uint64_t* C, const uint64_t* P, int gs, int bfirst,
                int ell, int nb, uint64_t* S, long sstride, hipStream_t s);

// select-and-sum of nq queries (client values Cq + q * cq_stride, NTT form [ell][2][L][N]) against
// nb plaintext batches; S entry of (batch b, query q) at (b * nq + q) * 2 L N.
void select_sum_multi(const Tables& T, const Consts& hc, const uint64_t* Cq, long cq_stride, const int* qslot,
                      int nq, const uint64_t* P, int gs, int bfirst, int ell, int nb, uint64_t* S,
                      hipStream_t s);

// The same on the int8 matrix cores, from digit planes (seven balanced base-256 digits per
// residue, code positions innermost in blocks of PL_K).  Plaintext planes of a 16-batch group:
// [L][N][kblocks][PL_DG][16][PL_K] int8; request planes of a query: [L][N][kblocks][PL_DG][2][PL_K]
// int8, query q's at Cp + qslot[q] * cps.  A tile is nb <= 64 batches: the group at Pp and the
// ones after it.  Valid for ell <= PL_MAX_ELL (exact int32 and 64-bit sums); rows
// b >= nb of a group are read but not written.
inline int plane_kblocks(int ell) { return (ell + PL_K - 1) / PL_K; }
size_t plaintext_plane_group_bytes(const Consts& hc, int ell);
size_t request_plane_bytes(const Consts& hc, int ell);
// group G (batches 16 G .. 16 G + 15) of a plaintext store with group size gs = 16
void plaintext_planes(const Tables& T, const Consts& hc, const uint64_t* P, int gs, int G, int ell, int8_t* out,
                      hipStream_t s);
// one query's NTT-form request [ell][2][L][N]
void request_planes(const Tables& T, const Consts& hc, const uint64_t* ch, int ell, int8_t* out, hipStream_t s);
void select_sum_planes(const Tables& T, const Consts& hc, const int8_t* Pp, const int8_t* Cp, long cps,
                       const int* qslot, int nq, int nb, int ell, uint64_t* S, hipStream_t s);
// The same over a run of ngroups consecutive 16-batch groups (nb <= 16 ngroups batches) in one
// launch, the request planes staged once per (l, k) and query octet in LDS: needs
// plane_kblocks(ell) <= PL_RUN_KBS (64.25 KB of LDS at 9 blocks).
constexpr int PL_RUN_KBS = 9;
void select_sum_planes_run(const Tables& T, const Consts& hc, const int8_t* Pp, int ngroups, const int8_t* Cp,
                           long cps, const int* qslot, int nq, int nb, int ell, uint64_t* S, hipStream_t s);

// acc[slot(q)] [L][L][N] += sum over b < nb of the relinearisation digits of the component-2
// rows c2[b * nq + q] ([L][N], cstride words apart): entry (i, j) adds [c2_i (Q/q_i)^-1]_{q_i}
// taken mod q_j (coefficient form).
void accumulate_digits(const Tables& T, const Consts& hc, const uint64_t* c2, long cstride, int nb, int nq,
                       const int* qslot, uint64_t* acc, long astride, hipStream_t s);

// ---------------- elementwise helpers ----------------
// p[0 .. words) = 0, and dst = src over words words, as kernels.
void zero_words(uint64_t* p, size_t words, hipStream_t s);
void copy_words(uint64_t* dst, const uint64_t* src, size_t words, hipStream_t s);
// out = a * b pointwise (both [rows][L][N] NTT form, b broadcast over rows if bcast)
void pointwise_mul(const Tables& T, const Consts& hc, const uint64_t* a, const uint64_t* b,
                   uint64_t* out, int rows, int nprimes, bool bcast, hipStream_t s);
// ct[c] *= k_c (per limb constants kq[L]) in place, both components ([2][L][N])
void scale_const(const Tables& T, const Consts& hc, uint64_t* ct, const uint64_t* kq, hipStream_t s);
// c0[l] += Delta_l * [m]_t (centred)  for a plaintext polynomial m (coefficient form)
void add_plain_poly(const Tables& T, const Consts& hc, uint64_t* ct, const uint32_t* m, hipStream_t s);
// encryption finish: c0 = Delta [m]_t - as - e, c1 = a    (count ciphertexts)
void encrypt_finish(const Tables& T, const Consts& hc, const uint32_t* m, const uint64_t* as,
                    const int32_t* e, const uint64_t* a, uint64_t* ct, int count, hipStream_t s);
// decryption: x = c0 + c1 s (coefficient form [count][L][N]) -> round(t x / Q) mod t
void decrypt_round(const Tables& T, const Consts& hc, const uint64_t* x, uint32_t* m, int count,
                   uint32_t* fallback_count, hipStream_t s);
// noise: max bit length of |[t x]_Q| over count ciphertext phases x -> atomicMax(out)
void noise_bits(const Tables& T, const Consts& hc, const uint64_t* x, int count, uint32_t* out,
                hipStream_t s);
// decryption phase in NTT form: x = c0 + c1 s; cth [count][2][L][N], sh [L][N], x [count][L][N]
void phase_ntt(const Tables& T, const Consts& hc, const uint64_t* cth, const uint64_t* sh, uint64_t* x,
               int count, hipStream_t s);
// relinearisation key finish: rlk_i0 = (Q/q_i) s^2 - a_i s - e_i, rlk_i1 = a_i
void keygen_finish(const Tables& T, const Consts& hc, const uint64_t* s2, const uint64_t* as,
                   const int32_t* e, const uint64_t* a, uint64_t* rlk, hipStream_t s);
// elementwise (a + b) mod q_l, rows [rows][nprimes][N]
void add_rows(const Tables& T, const Consts& hc, const uint64_t* a, const uint64_t* b, uint64_t* out,
              int rows, int nprimes, hipStream_t s);

// ---------------- measurement ----------------
// Lane operations per second of one VALU instruction kind on the current device (0
// v_mad_u64_u32, 1 v_mul_hi_u32, 2 v_mul_lo_u32, 3 v_add_u32, 4 v_mad_u32_u24, 5 v_fma_f64);
// synchronous; 0 or a negative status.
int probe_valu(int kind, double* lane_ops_per_s);

}  // namespace pepsi
