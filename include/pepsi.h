/*
 * pepsi.h -- C-ABI of the MI355X (gfx950) implementation of the server
 * computation of PEPSI PSI-cardinality (Mahdavi, Lukas, Kerschbaum et al.,
 * "PEPSI: Practically Efficient Private Set Intersection in the Unbalanced
 * Setting", arXiv 2310.14565).
 *
 * The calls follow the paper's statement of the protocol (Sec. 4):
 *   parameters and keys  ->  client preparation (Alg. 6, ClientDataPrep:
 *   hashing, constant-weight encoding, batching, encryption)  ->  server
 *   preparation (Alg. 6, ServerDataPrep)  ->  server computation (Alg. 1
 *   Arith-CW-Eq inside Alg. 2 Intersect / Alg. 5 PSI-Sum with unit values,
 *   i.e. PSI-Cardinality)  ->  result extraction (Alg. 3 / Alg. 5 decrypt).
 * Single evaluator steps (NTT, batching, select-and-sum, ciphertext product,
 * relinearisation) are exported too so that each can be checked on its own.
 *
 * Conventions
 *   - Ring R = Z[X]/(X^N + 1), N = 2^log_n; plaintext modulus t = 65537.
 *   - Ciphertext modulus Q = q_0 ... q_{L-1}: the L largest primes below 2^54
 *     with q = 1 mod 2N, in descending order.
 *   - A polynomial mod Q is limb-major: uint64 [L][N], residues in [0, q_l).
 *     A ciphertext is [2][L][N] (c0 then c1); a product before
 *     relinearisation is [3][L][N].  Every ciphertext crossing this boundary
 *     is in COEFFICIENT form.
 *   - Slots: slot k of a plaintext is its value at psi_t^(2k+1) (natural
 *     order), psi_t a primitive 2N-th root of unity mod t.  Plaintext
 *     polynomials are uint32 [N] with coefficients in [0, t); when a
 *     plaintext enters the ciphertext ring it is lifted to its centred
 *     representative in (-t/2, t/2].
 *   - Randomness is never drawn inside the library: the caller passes the
 *     secret key, the uniform polynomials and the errors.
 *   - "d_" arguments are device pointers on the library's current HIP device,
 *     "stream" is a hipStream_t (NULL = the default stream).  Device work is
 *     enqueued on the stream and the call returns; results are ready when the
 *     stream is synchronised.  Calls named "*_sync" or returning host values
 *     synchronise the stream themselves.
 *   - The caller owns every buffer it passes; the library owns its handles
 *     and the device memory behind them until the matching *_destroy.
 *   - Every function returns PEPSI_OK (0) or a negative pepsi_status; the
 *     thread's last message is in pepsi_last_error().  A protocol failure
 *     (cuckoo insertion or server bin overflow) is an error, never a silently
 *     wrong answer.
 */
#ifndef PEPSI_H
#define PEPSI_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PEPSI_OK = 0,
  PEPSI_E_ARG = -1,          /* null or inconsistent argument                          */
  PEPSI_E_PARAMS = -2,       /* unsupported parameters (N, L, h, code length, ...)     */
  PEPSI_E_CUCKOO = -3,       /* client insertion needs more evictions than allowed
                                (cuckoo hashing without a stash, Sec. 3.3 / 4.1)       */
  PEPSI_E_BIN_OVERFLOW = -4, /* a server bin holds more than mu elements (Sec. 4.1)    */
  PEPSI_E_RANGE = -5,        /* item out of range or duplicated                        */
  PEPSI_E_NOMEM = -6,        /* device or host allocation failed                       */
  PEPSI_E_DEVICE = -7        /* a HIP call failed (message names it)                   */
} pepsi_status;

/* Message of the calling thread's last failure ("" if none). */
const char* pepsi_last_error(void);

/* ------------------------------------------------------------------ */
/* Parameters (Table "notation"; eq. (1) for the code length)          */
/* ------------------------------------------------------------------ */
typedef struct pepsi_params pepsi_params;

typedef struct {
  uint32_t log_n;          /* N = 2^log_n = number of bins b; 10..14                   */
  uint32_t n_q;            /* L, number of ciphertext primes; 1..8                     */
  uint32_t h;              /* Hamming weight of the constant-weight code; 1..16        */
  uint32_t item_bits;      /* element bit length lambda; 1..64 (values above 32 bits:
                              large elements hashed to lambda bits, with the *64 calls) */
  uint32_t mu;             /* server maximum bin load                                  */
  uint32_t n_hash;         /* number of hash functions k (3 in the paper)             */
  uint32_t max_evictions;  /* cuckoo eviction limit per insertion                     */
  uint32_t flags;          /* 0 or PEPSI_PARAMS_PBH                                    */
  uint64_t hash_seed;      /* seed of the hash functions H_1..H_k                      */
} pepsi_params_desc;

/* Permutation-based hashing (Sec. 3.3): an element x = x_H || x_L (|x_H| = log_n) is
 * placed by hash function i in bin x_H ^ H_i(x_L) and stored as the shorter value
 * (i - 1) 2^(lambda - log_n) + x_L; the code length follows from the stored length
 * lambda_bar = lambda - log_n + ceil(log2 k) (the hash index is part of the value, so
 * that equal values in equal bins mean equal elements with k > 1 hash functions).
 * Needs item_bits > log_n. */
#define PEPSI_PARAMS_PBH 1u

#define PEPSI_MAX_PRIMES 17

typedef struct {
  uint32_t n, n_q, n_aux;  /* N, L and the auxiliary primes K used inside products      */
  uint32_t h, ell, mu;     /* ell = code length from eq. (1)                           */
  uint32_t item_bits, n_hash;
  uint64_t t;              /* 65537                                                    */
  uint64_t primes[PEPSI_MAX_PRIMES];  /* q_0..q_{L-1}, then the K auxiliary primes     */
  uint64_t psi[PEPSI_MAX_PRIMES];     /* primitive 2N-th roots used by the NTTs        */
  uint32_t psi_t;          /* primitive 2N-th root mod t defining the slot order       */
  uint32_t q_bits;         /* bit length of Q                                          */
  uint64_t query_bytes;    /* ell * 2 * L * N * 8: one client request                  */
  uint64_t ct_bytes;       /* 2 * L * N * 8                                            */
  uint64_t rlk_bytes;      /* L * 2 * L * N * 8                                        */
  uint64_t cache_bytes;    /* mu * ell * L * N * 8: the server plaintexts in NTT form  */
  uint32_t effective_bits; /* lambda_bar: bit length of the stored (encoded) values     */
  uint32_t flags;          /* as in the descriptor                                     */
} pepsi_params_info;

/* Creates a parameter set on the current HIP device: primes, NTT tables and RNS
 * constants are built on the host and copied to device memory owned by the
 * handle.  Errors: PEPSI_E_ARG (null), PEPSI_E_PARAMS (ranges above, or a code
 * length above 65534), PEPSI_E_NOMEM / PEPSI_E_DEVICE. */
int pepsi_params_create(const pepsi_params_desc* desc, pepsi_params** out);
int pepsi_params_get_info(const pepsi_params* params, pepsi_params_info* out);
void pepsi_params_destroy(pepsi_params* params);
/* Number of coefficients that took the exact multiword path of a rounding
 * decision (base extension, rescale, decryption) since the handle was created;
 * diagnostic only.  Synchronises the device. */
int pepsi_exact_path_count(const pepsi_params* params, uint64_t* out);

/* ------------------------------------------------------------------ */
/* Client preparation (Alg. 6 ClientDataPrep), host memory             */
/* ------------------------------------------------------------------ */
/* Cuckoo hashing of m distinct items (< 2^item_bits) into N bins with the
 * hash functions H_i(x) = mix64(x ^ (seed + i * 0x9E3779B97F4A7C15)) mod N,
 * i = 1..k, mix64 the SplitMix64 finaliser; an evicted element moves on to its
 * next hash function cyclically (Sec. 3.3).  table [N] receives the item of
 * each bin (with PEPSI_PARAMS_PBH its stored PBH value), valid [N] 1 for a real
 * item and 0 for a dummy.
 * Errors: PEPSI_E_RANGE (duplicate / out of range), PEPSI_E_CUCKOO. */
int pepsi_client_table(const pepsi_params* params, const uint32_t* items, uint64_t m,
                       uint32_t* table, uint8_t* valid);
/* Constant-weight encoding (Sec. 3.2, perfect mapping read as the
 * combinatorial number system) of a binned table and batching across bins:
 * planes [ell][N], planes[j][k] = 1 iff bit j of the codeword of bin k is set
 * (dummies encode to the all-zero word).  These are the slot vectors of the
 * ell client plaintexts pt_c[j]. */
int pepsi_codeword_planes(const pepsi_params* params, const uint32_t* table,
                          const uint8_t* valid, uint32_t* planes);

/* The same for elements and stored values of up to 64 bits (item_bits > 32, or stored PBH
 * values above 32 bits): items uint64 [m], table uint64 [N].  The 32-bit calls above reject
 * parameters whose stored values exceed 32 bits (PEPSI_E_ARG). */
int pepsi_client_table64(const pepsi_params* params, const uint64_t* items, uint64_t m,
                         uint64_t* table, uint8_t* valid);
int pepsi_codeword_planes64(const pepsi_params* params, const uint64_t* table,
                            const uint8_t* valid, uint32_t* planes);

/* ------------------------------------------------------------------ */
/* Large elements (Sec. 5, "Optimization for Large Elements", Lemma    */
/* "fail-collide"; Sec. 7, "Parameters for Large Elements"), host      */
/* ------------------------------------------------------------------ */
/* Element length for a failure rate below 2^-alpha: unequal elements hashed to lambda bits
 * match only if they collide and share a bin, and at most n_bins * mu_client * mu_server pairs
 * are compared, so *bits = lambda = alpha + ceil(log2(n_bins mu_client mu_server)) (alpha = 40
 * and mu_client = 1 in the paper's runs).  Needs no device.  Errors: PEPSI_E_ARG (a zero size). */
int pepsi_large_element_bits(uint32_t n_bins, uint32_t mu_client, uint32_t mu_server, uint32_t alpha,
                             uint32_t* bits);
/* Hashes count byte strings (element e is data[offsets[e] .. offsets[e + 1]), offsets has
 * count + 1 entries) to bits-bit values, 1 <= bits <= 64: out[e] = the first `bits` bits of
 * SHA-256 (FIPS 180-4) of the element, read big-endian (the paper names no hash function).  The
 * values are then the elements of pepsi_client_table64 / pepsi_server_create64 with
 * item_bits = bits.  Host memory; needs no device.  Errors: PEPSI_E_ARG. */
int pepsi_hash_elements(uint32_t bits, const uint8_t* data, const uint64_t* offsets, uint64_t count,
                        uint64_t* out);

/* ------------------------------------------------------------------ */
/* Keys, encryption, decryption (FV, Sec. 3.1), device memory          */
/* ------------------------------------------------------------------ */
/* Secret-key encryption of count slot vectors (Alg. 6):
 *   ct = ([-(a s + e) + Delta [m]_t]_Q, a),  m = encode(slots), Delta = floor(Q / t).
 * d_sk int8 [N] in {-1,0,1}; d_slots uint32 [count][N] (values mod t);
 * d_a uint64 [count][L][N] uniform residues; d_e int32 [count][N];
 * d_ct uint64 [count][2][L][N]. */
int pepsi_encrypt(const pepsi_params* params, const int8_t* d_sk, const uint32_t* d_slots,
                  const uint64_t* d_a, const int32_t* d_e, uint32_t count, uint64_t* d_ct,
                  void* stream);
/* Relinearisation key with the RNS gadget (the paper relies on its library's
 * relinearisation and does not describe it):
 *   rlk_i = ([-(a_i s + e_i) + (Q/q_i) s^2]_Q, a_i),  i in [L].
 * d_a uint64 [L][L][N], d_e int32 [L][N], d_rlk uint64 [L][2][L][N]. */
int pepsi_keygen_relin(const pepsi_params* params, const int8_t* d_sk, const uint64_t* d_a,
                       const int32_t* d_e, uint64_t* d_rlk, void* stream);
/* Decryption and decoding: slots = decode([round(t/Q [c0 + c1 s]_Q)]_t).
 * d_ct [count][2][L][N] -> d_slots uint32 [count][N] in [0, t). */
int pepsi_decrypt(const pepsi_params* params, const int8_t* d_sk, const uint64_t* d_ct,
                  uint32_t count, uint32_t* d_slots, void* stream);
/* Invariant-noise budget in bits of one ciphertext:
 *   bitlen(Q) - bitlen(max_k |[t (c0 + c1 s)]_Q|_k) - 1   (decryption is correct iff > 0).
 * Synchronises the stream; *budget is a host int. */
int pepsi_noise_budget(const pepsi_params* params, const int8_t* d_sk, const uint64_t* d_ct,
                       int32_t* budget, void* stream);

/* ------------------------------------------------------------------ */
/* Server preparation and computation (Alg. 6 ServerDataPrep; Alg. 1,  */
/* 2 and 5)                                                            */
/* ------------------------------------------------------------------ */
typedef struct pepsi_server pepsi_server;

#define PEPSI_SERVER_CACHE_PLAINTEXTS 1u  /* keep every server plaintext in NTT form in HBM */
#define PEPSI_SERVER_PLANES_ONLY 2u       /* with CACHE_PLAINTEXTS: keep them only as int8 digit
                                             planes (7/8 of the bytes), for servers that mostly
                                             batch or serve many queries                         */

typedef struct {
  uint32_t mu;             /* batches of the table                                     */
  uint32_t max_load;       /* fullest bin; batches at or above it hold only dummies    */
  uint32_t cached;         /* 1 if a plaintext cache is resident                       */
  uint32_t cached_batches; /* server batches whose plaintexts are cached (the first ones) */
  uint64_t device_bytes;   /* device memory held by the handle                         */
  uint32_t plane_groups;   /* cached 16-batch groups also held as int8 digit planes     */
} pepsi_server_info;

/* Server preparation: each of the n distinct items (< 2^item_bits) is appended to
 * each distinct bin among H_1..H_k (input order inside a bin), bins are padded to
 * mu with dummies, every entry is constant-weight encoded, and the codeword
 * positions uint16 [mu][N][h] (0xFFFF for dummies) are copied to device memory
 * owned by the handle.  With PEPSI_SERVER_CACHE_PLAINTEXTS the server plaintexts
 * pt_s[i'][j] are also batch-encoded and transformed into NTT form once, here
 * (ell * L * N * 8 bytes of HBM per server batch), for the first batches that fit
 * beside a 48 GiB working reserve (whole 16-batch tiles unless all fit; batches
 * holding only dummies are never stored); every evaluation regenerates the rest.
 * When the cache is kept in 16-batch groups and a second copy fits beside the same
 * reserve, the cached groups are also stored as int8 digit planes (seven balanced
 * base-256 digits per residue, about 7/8 of the cache's bytes), which the batched and
 * served evaluations contract on the matrix cores; pepsi_server_info.plane_groups
 * gives their number.  With PEPSI_SERVER_PLANES_ONLY as well, the NTT-form cache is not
 * kept: each 16-batch group is generated into a one-group staging store, converted to
 * digit planes and dropped, for as many groups as fit beside the reserve (so more batches
 * fit).  Every evaluation then also takes single queries through the planes, except
 * ranges that do not start at a multiple of 16 batches, which regenerate their plaintexts;
 * an evaluation fails with PEPSI_E_NOMEM if the request planes of its queries do not fit.
 * Results are identical in every mode.  Unknown flags, or PLANES_ONLY without
 * CACHE_PLAINTEXTS: PEPSI_E_ARG.
 * Synchronises the stream.  Errors: PEPSI_E_RANGE, PEPSI_E_BIN_OVERFLOW,
 * PEPSI_E_NOMEM. */
int pepsi_server_create(const pepsi_params* params, const uint32_t* items, uint64_t n,
                        uint32_t flags, void* stream, pepsi_server** out);
/* Server preparation with server values (Alg. 4 labelled PSI, Alg. 5 PSI-Sum): as
 * pepsi_server_create, where values[e] < t belongs to items[e] (host arrays of n).  The
 * value plaintext val_s[i'] of every batch that holds items (slot k = the value of the item
 * at entry (i', k) of the table, 0 for dummies) is batch-encoded and transformed into NTT
 * form here, [max_load][L][N] uint64 in HBM owned by the handle.  Every evaluation of the
 * handle (single, range, batched, served) then multiplies each batch's equality ciphertext
 * by val_s[i'] before the sum: with a mask the output is PSI-Sum (the decrypted slots sum
 * to the sum of the values of the common items, mod t); without one it is labelled PSI
 * (decrypted slot k = the value of the matched item in bin k, 0 if none, so labels should
 * be non-zero).  values == NULL is pepsi_server_create.  Synchronises the stream.  Errors:
 * as pepsi_server_create; PEPSI_E_RANGE for a value >= t. */
int pepsi_server_create_with_values(const pepsi_params* params, const uint32_t* items,
                                    const uint32_t* values, uint64_t n, uint32_t flags, void* stream,
                                    pepsi_server** out);
/* Server preparation with a bound on the plaintext cache: as
 * pepsi_server_create_with_values (values may be NULL), where with
 * PEPSI_SERVER_CACHE_PLAINTEXTS at most max_cached server batches are cached (0: as many as
 * fit).  The count is then rounded down to whole 16-batch tiles unless it covers every batch
 * that holds items, and evaluations regenerate the batches past it, so results are the same
 * for every bound; the bound trades HBM held by the handle against evaluation time (the
 * server's preprocessing, reused over many queries, Sec. 4.1).  pepsi_server_info.cached_batches
 * reports the count kept.  Errors: as pepsi_server_create_with_values. */
int pepsi_server_create_ex(const pepsi_params* params, const uint32_t* items, const uint32_t* values,
                           uint64_t n, uint32_t flags, uint32_t max_cached, void* stream,
                           pepsi_server** out);
/* Server preparation for elements of up to 64 bits (large elements hashed with
 * pepsi_hash_elements): as pepsi_server_create_ex with items uint64 [n]. */
int pepsi_server_create64(const pepsi_params* params, const uint64_t* items, const uint32_t* values,
                          uint64_t n, uint32_t flags, uint32_t max_cached, void* stream,
                          pepsi_server** out);
int pepsi_server_get_info(const pepsi_server* server, pepsi_server_info* out);
/* Copy of the codeword-position table uint16 [mu][N][h] to host memory. */
int pepsi_server_codewords(const pepsi_server* server, uint16_t* out);
void pepsi_server_destroy(pepsi_server* server);

/* Server computation, PSI-Cardinality (Alg. 5 with unit server values) or the
 * indicator of Alg. 2 when d_mask is NULL (with server values, PSI-Sum or labelled PSI:
 * each e below is first multiplied by val_s[i'], see pepsi_server_create_with_values):
 *   for every server batch i':  S = sum_j ct_j (*) pt_s[i'][j]          (Alg. 1, h')
 *                               e = prod_{r in [h]} (S + Delta [-r]_t)  (balanced tree,
 *                                   relinearised after every product)
 *   out = [(h!)^-1]_t * sum_i' e  (+ Delta [encode(mask)]_t on c0 when d_mask != NULL).
 * d_cts uint64 [ell][2][L][N] (the client request), d_rlk [L][2][L][N],
 * d_mask uint32 [N] with sum = 0 mod t (or NULL), d_out [2][L][N]; all coefficient
 * form.  Workspace is allocated by the handle on first use and kept. */
int pepsi_server_eval(pepsi_server* server, const uint64_t* d_cts, const uint64_t* d_rlk,
                      const uint32_t* d_mask, uint64_t* d_out, void* stream);
/* The same over server batches [batch_begin, batch_end) only; with finalize = 0
 * the output is sum_i' e (no (h!)^-1, no mask).  Sums over disjoint ranges add
 * up to the full sum mod Q. */
int pepsi_server_eval_range(pepsi_server* server, const uint64_t* d_cts, const uint64_t* d_rlk,
                            uint32_t batch_begin, uint32_t batch_end, uint32_t finalize,
                            const uint32_t* d_mask, uint64_t* d_out, void* stream);

/* Batched server computation: nq queries (each with its own request, key and optional mask;
 * arrays of nq device pointers given in host memory, masks may be NULL or hold NULL entries)
 * are evaluated together, so that every streamed tile of server plaintexts serves all of
 * them.  Each output equals what pepsi_server_eval gives for that query alone, bit for bit.
 * nq <= PEPSI_MAX_BATCH.  Workspace grows with the largest nq seen and is kept. */
#define PEPSI_MAX_BATCH 256
int pepsi_server_eval_batch(pepsi_server* server, uint32_t nq, const uint64_t* const* d_cts,
                            const uint64_t* const* d_rlk, const uint32_t* const* d_masks,
                            uint64_t* const* d_out, void* stream);

/* Schedule of the batched evaluation.  Each field 0 means "automatic".
 *   tile_batches:  server batches per tile (16, 32 or 64): the request planes or values are
 *                  read once per tile, and a tile's workspace grows with tile_batches * nq;
 *   select_kernel: PEPSI_SELECT_PLANES (int8 matrix cores over digit planes, when the server
 *                  holds them) or PEPSI_SELECT_VALU (64-bit products on the vector units; not
 *                  for a server that keeps its plaintexts only as planes);
 *   graph:         PEPSI_GRAPH_ON (the whole launch sequence of a call -- every query's
 *                  admission, all tiles and every query's finish -- is captured once into a HIP
 *                  graph and replayed by later calls with the same buffers) or PEPSI_GRAPH_OFF
 *                  (kernels launched one by one).  While event timing is enabled
 *                  (pepsi_server_timing) the launches are eager, so that every select-and-sum
 *                  launch is timed.
 * "Automatic" takes the entry of the library's tuned table (measured by autotune.py beside the
 * library) for the parameter set and the smallest tuned batch size >= nq, and otherwise a rule:
 * the largest of 64 / 32 / 16 batches whose workspace fits beside an 8 GiB reserve with digit
 * planes (16 without), the planes whenever the server holds them, graphs on.  A tile size whose
 * workspace does not fit falls back to 16 batches.  Results are identical under every schedule. */
#define PEPSI_SELECT_PLANES 1u
#define PEPSI_SELECT_VALU 2u
#define PEPSI_GRAPH_ON 1u
#define PEPSI_GRAPH_OFF 2u
#define PEPSI_RUN_ON 1u
#define PEPSI_RUN_OFF 2u
#define PEPSI_SCHEDULE_DEFAULT 0u   /* source: the rule above            */
#define PEPSI_SCHEDULE_TUNED 1u     /* source: an entry of the tuned table */
#define PEPSI_SCHEDULE_CALLER 2u    /* source: pepsi_server_set_schedule   */
typedef struct {
  uint32_t tile_batches, select_kernel, graph;
  uint32_t run;            /* with the matrix cores: PEPSI_RUN_ON (the select-and-sum of a run of
                              tiles -- all batches when their outputs fit -- is one launch that
                              reads each query's request planes once; the tiles' product trees
                              then follow) or PEPSI_RUN_OFF (one select-and-sum launch per tile)  */
  uint32_t source;         /* out only (pepsi_server_get_schedule)                      */
  double tuned_ms_per_query; /* out only: the tuned entry's measured time, 0 if none      */
} pepsi_schedule;
/* Forces the schedule of later batched evaluations (fields 0 stay automatic); NULL returns to
 * the automatic schedule.  Errors: PEPSI_E_ARG (a value outside the lists above, or VALU on a
 * server that holds its plaintexts only as planes). */
int pepsi_server_set_schedule(pepsi_server* server, const pepsi_schedule* schedule);
/* The schedule a batched evaluation of nq queries takes (the tile size before any fallback). */
int pepsi_server_get_schedule(pepsi_server* server, uint32_t nq, pepsi_schedule* out);

/* ------------------------------------------------------------------ */
/* Request and response compression (the request / response sizes of  */
/* Table "dipsi-cpsi")                                                 */
/* ------------------------------------------------------------------ */
/* The c1 part of a secret-key ciphertext is the uniform polynomial a, so a request can
 * carry a 32-byte seed instead of its ell c1 polynomials (half the request).  Both sides
 * expand a_j for ciphertext index j: a_{j,l}[k] = W mod q_l, W = the 16 bytes at offset 16 k
 * of the ChaCha20 keystream (RFC 8439; key = seed as 8 little-endian words, nonce = (j, l, 0),
 * block counter from 0), read little-endian (bias below 2^-74).  Writes a_j, j in
 * [first, first + count), at d_out + (j - first) * out_stride words, each [L][N]
 * (out_stride = L * N for a plain array; 2 * L * N with d_out = d_cts + L * N fills the c1
 * halves of a request [ell][2][L][N]).  Errors: PEPSI_E_ARG. */
int pepsi_expand_uniform(const pepsi_params* params, const uint8_t* seed, uint32_t first, uint32_t count,
                         uint64_t* d_out, uint64_t out_stride, void* stream);
/* Modulus switching of a response to the first prime: d_out [2][N] =
 * [round(q_0 X / Q)]_{q_0} for the centred lift X of every coefficient of d_ct [2][L][N]
 * (coefficient form), computed exactly; it decrypts under q_0 alone (a quarter of the
 * response at L = 4). */
int pepsi_mod_switch(const pepsi_params* params, const uint64_t* d_ct, uint64_t* d_out, void* stream);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching over one prepared server               */
/* ------------------------------------------------------------------ */
/* A serving handle runs a worker thread with its own HIP stream.  The server
 * batches are walked as a circular sequence of 16-batch tiles; every step runs one
 * tile for all admitted queries, so each streamed plaintext tile serves all of
 * them.  A submitted request waits in a queue until a query slot is free, is
 * admitted at the next step boundary, and completes after one full cycle of tiles
 * (its result is bit-identical to pepsi_server_eval on the same inputs).  The
 * number of slots is max_active (0: PEPSI_MAX_BATCH), capped by hbm_budget / (device
 * bytes per slot, pepsi_serve_info.slot_bytes) when hbm_budget is non-zero: requests are
 * admitted by memory, and the rest wait.  The handle's workspace is allocated at creation.
 * The worker keeps up to two steps in flight on the device and completes requests from
 * events, so its host bookkeeping overlaps the device's work.
 * Device buffers of a request must be ready (their producing work synchronised)
 * at submission and stay valid until it completes.  submit / poll / wait /
 * get_info are thread-safe.  Times are seconds on pepsi_clock(), a monotonic
 * clock. */
typedef struct pepsi_serve pepsi_serve;
typedef struct {
  double submit_s, admit_s, done_s;
  uint32_t slot, done;
} pepsi_req_stats;
typedef struct {
  uint32_t slots, tiles, active, queued;
  uint64_t steps, completed;
  uint64_t slot_bytes;     /* device bytes one query slot takes (the admission unit)     */
} pepsi_serve_info;
double pepsi_clock(void);
int pepsi_serve_create(pepsi_server* server, uint32_t max_active, uint64_t hbm_budget, pepsi_serve** out);
int pepsi_serve_submit(pepsi_serve* serve, const uint64_t* d_cts, const uint64_t* d_rlk,
                       const uint32_t* d_mask, uint64_t* d_out, uint64_t* req_id);
int pepsi_serve_poll(pepsi_serve* serve, uint64_t req_id, int* done, pepsi_req_stats* stats);
int pepsi_serve_wait(pepsi_serve* serve, uint64_t req_id, pepsi_req_stats* stats);
int pepsi_serve_get_info(pepsi_serve* serve, pepsi_serve_info* out);
/* Waits for every submitted request, then stops the worker and frees the handle. */
void pepsi_serve_destroy(pepsi_serve* serve);

/* Event timing of a server's evaluations, for measurement.  While enabled,
 * every select-and-sum launch (the kernel that streams the server plaintexts),
 * every forward and inverse transform of the request, the product tree and the
 * finish, every exact rescale and Q -> B extension of the product tree, and every whole
 * evaluation are bracketed by HIP events on the
 * evaluation's stream.  The call synchronises the device, folds finished event pairs into
 * the totals, then applies reset (zero the totals) and enable (1 on, 0 off). */
typedef struct {
  uint64_t select_sum_launches;
  uint64_t select_sum_bytes;   /* algorithmic bytes: plaintexts + client ciphertexts
                                  read once + sums written, per launch */
  double select_sum_ms;
  uint64_t evals;
  double eval_ms;
  uint64_t ntt_fwd_launches, ntt_fwd_rows;  /* the evaluations' forward transforms over Q or B */
  double ntt_fwd_ms;
  uint64_t ntt_inv_launches, ntt_inv_rows;  /* and their inverse transforms                   */
  double ntt_inv_ms;
  /* The exact rescales round(t d / Q) of the product tree (k_scale_round) and the exact Q -> B
   * extensions (k_ext_q_to_b, k_add_ext_q_to_b), with their 54-bit modular products: per
   * coefficient, a rescale takes L + K products y_p = d_p (P/p)^-1 (L + K more with the first
   * level's linear terms), K (L + 1) for the sums into B, K for their scaling and L (K + 1) for the
   * sums back into Q; an extension L + K (L + 1).  A product is one Shoup multiplication or one
   * term of an exact sum of products; each costs at least three 32 x 32 -> 64-bit multiply-adds
   * (27-bit halves). */
  uint64_t rescale_launches, rescale_products;
  double rescale_ms;
  uint64_t ext_launches, ext_products;
  double ext_ms;
} pepsi_timing;
int pepsi_server_timing(pepsi_server* server, int enable, int reset, pepsi_timing* out);

/* Issue rate of one vector-ALU instruction on the current device, in lane operations per
 * second: eight independent chains of the instruction per thread, 8 waves per SIMD on every
 * compute unit, timed with events (the measured peaks of the integer-VALU roofline).  kind: 0
 * v_mad_u64_u32, 1 v_mul_hi_u32, 2 v_mul_lo_u32, 3 v_add_u32, 4 v_mad_u32_u24, 5 v_fma_f64,
 * 6 v_mfma_i32_16x16x64_i8 (the digit-plane select-and-sum's matrix instruction; eight
 * independent accumulator chains per wave; the result is then in int8 operations per second,
 * 2 x 16 x 16 x 64 per wave instruction).
 * Synchronous; allocates and frees a small buffer.  Errors: PEPSI_E_ARG, PEPSI_E_DEVICE. */
int pepsi_probe_valu(uint32_t kind, double* lane_ops_per_s);

/* ------------------------------------------------------------------ */
/* Single evaluator steps                                              */
/* ------------------------------------------------------------------ */
/* Negacyclic NTT of rows [rows][N] in place; row r is taken modulo prime
 * (first_prime + r % n_primes) of the primes listed in pepsi_params_info.
 * Forward output order: out[k] = a(psi^(2 brv(k) + 1)) (bit-reversed); inverse
 * = its exact inverse.  Inputs must be reduced (< the row's prime). */
int pepsi_ntt(const pepsi_params* params, uint64_t* d_data, uint32_t rows, uint32_t first_prime,
              uint32_t n_primes, int inverse, void* stream);
/* Batch encoding over Z_t (Sec. 4.1, "batching"): slots [rows][N] -> plaintext
 * polynomials [rows][N], and back. */
int pepsi_encode(const pepsi_params* params, const uint32_t* d_slots, uint32_t rows,
                 uint32_t* d_poly, void* stream);
int pepsi_decode(const pepsi_params* params, const uint32_t* d_poly, uint32_t rows,
                 uint32_t* d_slots, void* stream);
/* Select-and-sum of one server batch (Alg. 1, first line, over all bins):
 *   out = sum_j ct_j (*) p_j,  p_j = encode(slots with slot k = [j in cw[k][0..h)]).
 * d_cts [ell][2][L][N], d_cw uint16 [N][h] (0xFFFF = no position), d_out [2][L][N]. */
int pepsi_select_sum(const pepsi_params* params, const uint64_t* d_cts, const uint16_t* d_cw,
                     uint64_t* d_out, void* stream);
/* FV ciphertext product without relinearisation (Sec. 3.1, "Multiplication"):
 *   out_k = [round(t/Q * (x (x) y)_k)]_Q,  x, y lifted to centred integers,
 *   (x (x) y) = (x0 y0, x0 y1 + x1 y0, x1 y1) over Z[X]/(X^N + 1).
 * d_x, d_y [2][L][N]; d_out [3][L][N]. */
int pepsi_multiply(const pepsi_params* params, const uint64_t* d_x, const uint64_t* d_y,
                   uint64_t* d_out, void* stream);
/* The product of pepsi_multiply, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): its scratch (the operands
 * extended to the auxiliary base and the tensor, 8 (4 L N + 4 K N + 3 (L + K) N) bytes) lives in a
 * fixed 8 MiB device array of the library, of which each GPU holds its own copy until the process
 * ends; the call allocates and frees nothing and does not synchronise.  Parameter sets whose
 * scratch exceeds 8 MiB (e.g. N = 16384 with 8 primes) are refused with PEPSI_E_ARG before any
 * device work; N = 8192 with 4 primes takes 4.1 MB.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (several streams or threads) race and must be serialised by the
 * caller.  Must run on the device the parameters were created on.  Same arguments and result as
 * pepsi_multiply. */
int pepsi_multiply_noalloc(const pepsi_params* params, const uint64_t* d_x, const uint64_t* d_y,
                           uint64_t* d_out, void* stream);
/* Relinearisation with the RNS gadget: digits D_i = [d2 (Q/q_i)^-1]_{q_i} in
 * [0, q_i); out = (d0 + sum_i D_i rlk_i0, d1 + sum_i D_i rlk_i1).
 * d_ct3 [3][L][N], d_rlk [L][2][L][N], d_out [2][L][N]. */
int pepsi_relin(const pepsi_params* params, const uint64_t* d_ct3, const uint64_t* d_rlk,
                uint64_t* d_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PEPSI_H */
