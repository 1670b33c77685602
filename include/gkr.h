/*
 * gkr.h -- C ABI of the MI355X GKR prover / verifier over F_p, p = 2^61 - 1.
 *
 * Method: Thaler, Roberts, Mitzenmacher, Pfister, "Verifiable Computation
 * with Massively Parallel Interactive Proofs" (GKR protocol, Sec. 3.1;
 * parallel prover, Sec. 4.1.1; verifier, Sec. 4.1.2; field, Sec. 6.1).
 *
 * Conventions shared by every entry point
 *   - Field elements are uint64_t in canonical form, 0 <= x < p.
 *   - Layers are numbered 0 = output ... d = input (the reverse of the
 *     paper's numbering).  Layer i < d has S_i gates; gate g has a type
 *     (GKR_ADD or GKR_MUL) and two wires in1[g], in2[g] into layer i+1.
 *     s_i = ceil(log2 S_i) (0 when S_i = 1); a wire may name a padding slot
 *     of layer i+1 (index < 2^{s_{i+1}}), whose value is 0.
 *   - Transcript layout ("msgs"): V_0[0..S_0) (the claimed outputs), then per
 *     layer i = 0..d-1: G_j(0), G_j(1), G_j(2) for each of the
 *     n_i = s_i + 2 s_{i+1} sum-check rounds (variables a, then b, then c,
 *     least significant bit first), then v1 = ~V_{i+1}(b*), v2 = ~V_{i+1}(c*),
 *     then h(t) = ~V_{i+1}(b* + t (c* - b*)) for t = 2 .. s_{i+1}.
 *     Challenges ("chals"): z_0 (s_0 values), then per layer r_1..r_{n_i}, tau.
 *   - Challenges come from SplitMix64 (Steele, Lea, Flood 2014) seeded with
 *     (seed << 8) | 2 (GKR) or (seed << 8) | 4 (F2 sum-check); a draw keeps
 *     the low 61 bits of an output and redraws on 2^61 - 1.  The prover reads
 *     challenge j only after message j is complete.
 *   - Buffers: every pointer is owned by the caller and is neither freed nor
 *     retained after the call returns.  "on_device" flags say whether a
 *     pointer is a device (HBM) address or host memory.  Transcript outputs
 *     are host memory.
 *   - Streams: hip_stream is a hipStream_t or NULL (the library's own
 *     stream on the current device).  Calls return after their work on that
 *     stream has finished.
 *   - Errors: every function returns GKR_OK (0) or a negative code;
 *     gkr_last_error() gives a message for the calling thread.  Rejection
 *     of a proof is not an error: gkr_verify returns GKR_OK, *accepted = 0.
 */
#ifndef GKR_H
#define GKR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GKR_OK = 0,
    GKR_ERR_INVALID = -1, /* malformed circuit, size or argument            */
    GKR_ERR_RANGE = -2,   /* an input value is not below p                  */
    GKR_ERR_NOMEM = -3,   /* host or device allocation failed               */
    GKR_ERR_DEVICE = -4,  /* a HIP runtime error                            */
    GKR_ERR_BUFSIZE = -5  /* a transcript buffer has the wrong length       */
};

enum { GKR_ADD = 0, GKR_MUL = 1 };

/* How the prover computes the rounds over the wire variables (b, c):
 *   GKR_OMEGA_GATES   every round is a pass over the layer's gates, each gate
 *                     contributing its term (Sec. 4.1.1), O(S log S) per layer;
 *   GKR_OMEGA_TABLES  the gates' weights are summed once per phase into
 *                     tables indexed by the bound wire, and every round folds
 *                     those tables (which halve each round), O(S + 2^{s'}).
 *                     The circuit's first layers whose tables all fit one
 *                     workgroup's LDS (2^{s_i}, 2^{s_{i+1}} <= 1024 values,
 *                     at most 32 gates on a wire) run whole in one launch,
 *                     their tables kept in LDS from one layer to the next
 *                     (not for GKR_MEM_LAYER circuits);
 *   GKR_OMEGA_TABLES_STEPWISE  the same tables, every layer in launches of
 *                     its own.
 * All give the same transcript bit for bit. */
enum { GKR_OMEGA_GATES = 0, GKR_OMEGA_TABLES = 1, GKR_OMEGA_TABLES_STEPWISE = 2 };

/* Reasons for rejection (gkr_reject_info.check). */
enum {
    GKR_CHECK_MALFORMED = 1, /* wrong length, or a value not below p          */
    GKR_CHECK_ROUND = 2,     /* G_j(0) + G_j(1) differs from the claim        */
    GKR_CHECK_WIRING = 3,    /* last claim of a layer differs from
                                beta(z,a*) [add~ (v1+v2) + mult~ v1 v2]        */
    GKR_CHECK_LINE = 4,      /* v1 != v2 although layer i+1 has one gate      */
    GKR_CHECK_INPUT = 5      /* final claim differs from the input's
                                multilinear extension at the last point       */
};

typedef struct gkr_circuit gkr_circuit; /* opaque; immutable after creation */

typedef struct {
    int32_t layer; /* layer whose check failed (-1: whole transcript)       */
    int32_t round; /* sum-check round within the layer, or -1               */
    int32_t check; /* GKR_CHECK_*                                           */
} gkr_reject_info;

/* Create a circuit (Sec. 3.1: layered, fan-in 2, ADD and MUL gates).
 *   num_layers   d + 1 >= 2, including the input layer.
 *   layer_sizes  [d+1] host array, S_0 (output) .. S_d (input), each >= 1
 *                and < 2^31.
 *   gate_type, in1, in2   [d] host arrays of host pointers; layer i's arrays
 *                have S_i entries (types GKR_ADD / GKR_MUL, wires
 *                < 2^{s_{i+1}}).
 * The arrays are validated and copied to device memory (struct-of-arrays
 * per layer); the caller may free them afterwards.
 * Errors: GKR_ERR_INVALID, GKR_ERR_NOMEM, GKR_ERR_DEVICE. */
int gkr_circuit_create(uint32_t num_layers, const uint32_t *layer_sizes,
                       const uint8_t *const *gate_type, const uint32_t *const *in1,
                       const uint32_t *const *in2, gkr_circuit **out);

/* Release a circuit and the device memory it holds (NULL is ignored).
 * No proof on the circuit may be running. */
void gkr_circuit_destroy(gkr_circuit *c);

/* Choose the omega-phase algorithm of a circuit (default GKR_OMEGA_TABLES).
 * Frees the circuit's proof scratch, which the next proof re-creates.
 * Must not be called while a proof on the circuit runs.
 * Errors: GKR_ERR_INVALID. */
int gkr_circuit_set_algorithm(gkr_circuit *c, int omega_algo);

/* Memory strategies for a circuit's proofs (Sec. 5.1.1 - 5.1.3).
 *   GKR_MEM_RESIDENT  "no copying": the gate arrays and every layer's
 *                     tables stay in device memory (the default).
 *   GKR_MEM_LAYER     "copy once per layer": the gate arrays and the gate
 *                     value tables V_i of all layers live in pinned host
 *                     memory; the device holds three value-table slots and
 *                     two gate-array slots sized for the widest layer, plus
 *                     the round tables.  Evaluation copies each V_i out as
 *                     it is written; layer i's sum-check reads V_i, V_{i+1}
 *                     and its gate groups from the slots while V_{i+2} and
 *                     layer i+1's groups are copied in on a second stream.
 *   GKR_MEM_MESSAGE   "copy every message": the gate arrays, value tables
 *                     and round tables all live in pinned host memory and
 *                     every round's kernels read and write them in place
 *                     through the host link, so each message moves its
 *                     layer's data again; the device holds only the small
 *                     per-proof state (eq half tables, partial rows,
 *                     transcript, step program).
 *   GKR_MEM_AUTO      the first of the three whose device bytes fit.
 * Transcripts do not depend on the mode.  Proofs in GKR_MEM_LAYER are
 * launched one by one (no graph replay) and cannot be batched; a server
 * runs a circuit that is not resident, or whose resident scratch exceeds
 * its budget, in GKR_MEM_MESSAGE. */
enum { GKR_MEM_RESIDENT = 0, GKR_MEM_LAYER = 1, GKR_MEM_MESSAGE = 2, GKR_MEM_AUTO = 3 };

/* Device and pinned host bytes one proof of c needs in a mode (RESIDENT,
 * LAYER or MESSAGE), counting the circuit's gate arrays where the mode puts
 * them; sized without allocating.  Errors: GKR_ERR_INVALID. */
int gkr_memory_need(gkr_circuit *c, int mode, uint64_t *device_bytes, uint64_t *host_bytes);

/* Choose how c's proofs place their data.  mode: one of GKR_MEM_*; with
 * device_budget_bytes > 0 the chosen mode's device bytes (gkr_memory_need)
 * must fit it (GKR_MEM_AUTO picks the first that does); 0 means no limit.
 * The gate arrays move to pinned host memory for LAYER and MESSAGE and back
 * to the device for RESIDENT; the circuit's proof scratch, cached batch plans
 * and servers' idle scratch for it are released.  *chosen (may be NULL)
 * receives the mode.  Must not be called while a proof on c runs.
 * Errors: GKR_ERR_INVALID, GKR_ERR_NOMEM (nothing fits, or an allocation
 * failed), GKR_ERR_DEVICE. */
int gkr_circuit_set_memory(gkr_circuit *c, int mode, uint64_t device_budget_bytes, int *chosen);

/* Transcript lengths for the layout above. */
int gkr_transcript_size(const gkr_circuit *c, uint64_t *n_msgs, uint64_t *n_chals);

/* Shape summary: total gates including inputs (as Table 2 counts them),
 * total sum-check rounds, and the number of layers d + 1. */
int gkr_circuit_info(const gkr_circuit *c, uint64_t *gates, uint64_t *rounds,
                     uint32_t *num_layers);

/* Prove (Sec. 3.1, 4.1.1): evaluate the circuit on `inputs` (S_d values,
 * each < p; device or host memory), then run one sum-check per layer.
 *   msgs   host array of exactly n_msgs values (gkr_transcript_size).
 *   chals  host array of n_chals values, or NULL.
 * Device scratch is allocated on the first call for a circuit and reused.
 * Errors: GKR_ERR_INVALID (NULL arguments), GKR_ERR_RANGE (an input >= p;
 * the transcript is then unspecified), GKR_ERR_NOMEM, GKR_ERR_DEVICE. */
int gkr_prove(const gkr_circuit *c, const uint64_t *inputs, int inputs_on_device, uint64_t seed,
              uint64_t *msgs, uint64_t *chals, void *hip_stream);

/* Verify (Sec. 2.2, 4.1.2): replay every round check, the per-layer wiring
 * identity, the line step, and compare the last claim with the inputs'
 * multilinear extension, computed on the device in one pass over the
 * inputs (host inputs stream through it in chunks of 2^23 values, so the
 * verifier holds two chunks on the device).  add~ and mult~ come from a
 * closed form on the host where the layer has one (gkr_circuit_wiring),
 * else from one pass over the layer's gates on the device.
 *   msgs/n_msgs   host transcript.  accepted: 1 or 0.  why: NULL or filled
 *   on rejection (layer/round/check as in gkr_reject_info).
 * Errors: GKR_ERR_INVALID, GKR_ERR_RANGE (an input >= p), GKR_ERR_NOMEM,
 * GKR_ERR_DEVICE.  A wrong-length or non-canonical transcript is a
 * rejection (GKR_CHECK_MALFORMED), not an error. */
int gkr_verify(const gkr_circuit *c, const uint64_t *inputs, int inputs_on_device, uint64_t seed,
               const uint64_t *msgs, uint64_t n_msgs, int *accepted, gkr_reject_info *why,
               void *hip_stream);

/* Wiring shapes (Sec. 3.1's add~ and mult~ at a point (a, b, c)).  At
 * creation every layer whose gates are all ADD or all MUL is matched against
 * shapes whose predicate W(a, b, c) = sum_g chi_g(a) chi_in1(g)(b)
 * chi_in2(g)(c) is a product over the bits of g; the verifier evaluates
 * those in O(s_i + s_{i+1}) field operations on the host:
 *   GKR_WIRING_TREE     gate g reads 2g and 2g + 1 (the binary sum trees);
 *   GKR_WIRING_SQUARE   gate g reads g twice (F2's squares, F0's squaring);
 *   GKR_WIRING_MATMULT  S = N^3 (N a power of two), gate (iN + j)N + k
 *                       reads iN + k and N^2 + kN + j (A then B row-major).
 * Any other layer is GKR_WIRING_GATES (one pass over its gates).
 * gkr_circuit_wiring: the shape of layer `layer` (0 <= layer < d).
 * Errors: GKR_ERR_INVALID. */
enum { GKR_WIRING_GATES = 0, GKR_WIRING_TREE = 1, GKR_WIRING_SQUARE = 2, GKR_WIRING_MATMULT = 3 };
int gkr_circuit_wiring(const gkr_circuit *c, uint32_t layer, int *form);
/* Use the closed forms in later gkr_verify calls of this process (enable 1,
 * the default) or pass over every layer's gates (0); returns the previous
 * setting.  Verdicts do not depend on it. */
int gkr_verify_closed_forms(int enable);

/* Launch shapes.  A grid step over U work items (gates, wires, table
 * entries or quads of them) launches ceil(U / (512 q)) workgroups of 512
 * threads, at most `cap`, where q (items per thread: 1, 2, 4, 8) and cap
 * (256, 512, 1024, 2048) are chosen per step kind and size class (ceil
 * log2 U).  gkr_autotune proves each of the n circuits (inputs as in
 * gkr_prove, seeds 1..reps) under each of the 16 shapes, timing every grid
 * launch with events (one warm-up proof per shape), and keeps for each
 * (kind, class) met the fastest shape; plans made afterwards, including
 * cached batch plans and a server's idle scratch, use it.  Transcripts do
 * not depend on the shapes (the sums are exact).  Not safe to call while
 * other threads prove on the same circuits.  Errors: GKR_ERR_INVALID,
 * GKR_ERR_RANGE, GKR_ERR_NOMEM, GKR_ERR_DEVICE. */
int gkr_autotune(uint32_t n, const gkr_circuit *const *circuits, const uint64_t *const *inputs,
                 int inputs_on_device, uint32_t reps, void *hip_stream);
/* The shape table as bytes, to keep a tuning across processes: with buf
 * NULL, *len receives the size; otherwise *len is the buffer size (at
 * least that) and receives it.  Errors: GKR_ERR_INVALID, GKR_ERR_BUFSIZE. */
int gkr_tune_get(uint8_t *buf, uint32_t *len);
/* Restore a table from gkr_tune_get (buf NULL: back to the defaults).
 * Errors: GKR_ERR_INVALID (not a table of this library). */
int gkr_tune_set(const uint8_t *buf, uint32_t len);

/* Batched proving: n proofs advance together, one launch per step running
 * that step of every proof still going (one workgroup range per proof), so a
 * batch costs as many launches as its longest proof has steps.  With
 * GKR_BATCH_GRAPH the launch sequence is captured once as a HIP graph and
 * replayed by later calls over the same circuits.  Each proof's transcript is
 * bit for bit the one gkr_prove returns for the same circuit, inputs and seed.
 *   circuits  n handles (a handle may repeat); inputs: n device pointers of
 *             S_d values (inputs_on_device must be 1); seeds: n seeds;
 *   msgs      n host arrays of each circuit's n_msgs values.
 * The plan (scratch per entry, schedule, graph) of the last few distinct
 * circuit lists is cached; destroying a circuit drops the plans using it.
 * Errors: GKR_ERR_INVALID, GKR_ERR_RANGE, GKR_ERR_NOMEM, GKR_ERR_DEVICE. */
enum { GKR_BATCH_GRAPH = 1 };
int gkr_batch_prove(uint32_t n, const gkr_circuit *const *circuits, const uint64_t *const *inputs,
                    int inputs_on_device, const uint64_t *seeds, uint64_t *const *msgs, int flags,
                    void *hip_stream);

/* Serving: a proof server with continuous batching.  A scheduler thread
 * keeps up to max_slots proofs in flight; every launch runs the next step of
 * each of them, so requests that arrive while others run join at the next
 * launch.  A request is admitted when a slot is free and its device scratch
 * fits hbm_budget_bytes (idle scratch is pooled per circuit and reused).
 * Results are bit for bit those of gkr_prove.
 *   gkr_server_create   max_slots in [1, 127].
 *   gkr_server_submit   copies the S_d host inputs (each < p); the circuit
 *                       must outlive the request.  *req_id identifies it.
 *   gkr_server_poll     *done = 1 once finished; then copies the transcript
 *                       into msgs (n_msgs values, may be NULL), sets
 *                       *latency_s (submission to completion) and forgets
 *                       the request.
 *   gkr_server_stats    proofs in flight, queued requests, scratch bytes held.
 *   gkr_server_destroy  waits for the scheduler; pending requests are dropped.
 * Errors: GKR_ERR_INVALID, GKR_ERR_RANGE, GKR_ERR_NOMEM, GKR_ERR_DEVICE. */
typedef struct gkr_server gkr_server;
int gkr_server_create(uint64_t hbm_budget_bytes, uint32_t max_slots, gkr_server **out);
int gkr_server_submit(gkr_server *s, const gkr_circuit *c, const uint64_t *inputs, uint64_t seed,
                      uint64_t *req_id);
int gkr_server_poll(gkr_server *s, uint64_t req_id, uint64_t *msgs, int *done, double *latency_s);
int gkr_server_stats(gkr_server *s, uint32_t *running, uint32_t *queued, uint64_t *hbm_used);
void gkr_server_destroy(gkr_server *s);

/* Sum-check for F2 = sum_x ~a(x)^2 over {0,1}^l, n = 2^l (the sum-check
 * primitive, Sec. 7, on the second frequency moment of Sec. 3.2).
 *   freq   n uint32 values (device or host); n a power of two, n <= 2^32.
 *   msgs   host array of 1 + 3 l values: F2, then G_j(0), G_j(1), G_j(2)
 *          for rounds j = 1..l (G_j(t) = sum_m ((1-t) A[2m] + t A[2m+1])^2
 *          over the table A folded by the earlier challenges).
 *   chals  host array of l values, or NULL.
 * Errors: GKR_ERR_INVALID, GKR_ERR_NOMEM, GKR_ERR_DEVICE. */
int f2_sumcheck_prove(const uint32_t *freq, uint64_t n, int on_device, uint64_t seed,
                      uint64_t *msgs, uint64_t *chals, void *hip_stream);

/* Verify an F2 sum-check transcript: round checks, then the last claim
 * against ~a(r)^2 with ~a(r) computed on the device from freq.
 * Rejections: GKR_CHECK_MALFORMED, GKR_CHECK_ROUND, GKR_CHECK_INPUT. */
int f2_sumcheck_verify(const uint32_t *freq, uint64_t n, int on_device, uint64_t seed,
                       const uint64_t *msgs, uint64_t n_msgs, int *accepted,
                       gkr_reject_info *why, void *hip_stream);

/* f2_sumcheck_prove without any allocation, for callers that cannot
 * allocate device or pinned memory during a call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, transcript and errors as f2_sumcheck_prove, with n <= 2^22:
 * its scratch is one static 48 MiB device array per GPU (the two folded
 * tables, the partial rows, the transcript and, for host inputs, their
 * staging copy), held from the library's load on that GPU until the
 * process ends; larger n returns GKR_ERR_NOMEM.  msgs and chals are copied
 * straight into the caller's host arrays.  Calls on one GPU share the
 * array: calls from this process are serialised by a lock, and calls that
 * overlap on one GPU from elsewhere (another process's graph replaying
 * it) race. */
int f2_sumcheck_prove_noalloc(const uint32_t *freq, uint64_t n, int on_device, uint64_t seed,
                              uint64_t *msgs, uint64_t *chals, void *hip_stream);

/* Non-interactive F2 (Sec. 3.2; GPU version Sec. 4.2; Table 3):
 * a streaming verifier keeping v field words, a proof of 2h words.  The n
 * values a (each below p; host, or device if on_device) fill a v x h grid,
 * v = ceil(n / h), cell (row y, column j) = a[j v + y] (zero past n).  h
 * must be odd, divide (p - 1) / 2 and have prime factors among 3, 5, 7, 11,
 * 13 with 3 and 5 at most squared (e.g. 45, 585, 1287, 2475, 5005).  Row y
 * is the polynomial f_y of degree < h through the order-h subgroup of
 * F_p^* (generator 37^((p-1)/h)); the proof msgs[k] = sum_y f_y(xi^k)^2,
 * k < 2h, xi = 37^((p-1)/(2h)), so F2 = sum_j msgs[2j].  msgs: 2h words,
 * caller-owned host memory.  Errors: GKR_ERR_INVALID (NULL, n = 0,
 * unsupported h), GKR_ERR_RANGE (a value not below p), GKR_ERR_DEVICE. */
int nif2_prove(const uint64_t *a, uint64_t n, uint32_t h, int on_device, uint64_t *msgs,
               void *hip_stream);

/* The verifier: its secret r is drawn from SplitMix64 (seed, purpose 9)
 * before the stream is read; it keeps f_y(r) for every row and accepts iff
 * the polynomial through the 2h proof values equals sum_y f_y(r)^2 at r.
 * *f2 (may be NULL) receives sum_j msgs[2j].  A proof of the wrong length
 * or with a value not below p is rejected (*accepted = 0, GKR_OK).
 * Errors: as nif2_prove. */
int nif2_verify(const uint64_t *a, uint64_t n, uint32_t h, int on_device, uint64_t seed,
                const uint64_t *msgs, uint64_t n_msgs, int *accepted, uint64_t *f2,
                void *hip_stream);

/* F_p arithmetic on the device field module (Sec. 6.1), for checking it:
 * out[k] = a[k] op b[k], op 0 = add, 1 = sub, 2 = mul; op 3 = the sum of
 * the 64 products a[j] b[j], j = k, k+1, ..., k+63 (indices mod n),
 * accumulated in 128 bits and reduced once (the lazy reduction the prover's
 * sums use); op 4 = a[k] b[k]^256 by 256 successive products (independent
 * chains over k: a probe of the product rate).  a, b, out are device arrays
 * of n canonical values.  Errors: GKR_ERR_INVALID, GKR_ERR_DEVICE. */
int gkr_field_op(int op, const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n,
                 void *hip_stream);

/* Per-kernel timing.  While enabled (flag 1, or 2 to also keep every
 * launch's record), every launch of the prover's kernels is bracketed by
 * HIP events on its stream (single proofs then run launch by launch, and
 * batches without their graph).  gkr_profile_read synchronises, then
 * reports for each kernel class k < *n_classes: total milliseconds, launch
 * count, algorithmic bytes moved and algorithmic 64 x 64-bit modular
 * products (the per-unit figures of each kernel times the units processed),
 * and resets the totals.  names, ms, launches, bytes, mods may be NULL;
 * names receives static strings.  Errors: GKR_ERR_INVALID, GKR_ERR_DEVICE. */
int gkr_profile_enable(int flag);
int gkr_profile_read(uint32_t *n_classes, const char **names, double *ms, uint64_t *launches,
                     double *bytes, double *mods);
/* The launches kept since the last call (flag 2): with every output NULL,
 * *n receives their number; otherwise *n is the room and receives the
 * number, and launch k's class, size class (ceil log2 of its work items,
 * -1 for steps not sized by work items), milliseconds, bytes and products
 * are written; the records are then dropped.  Errors: GKR_ERR_INVALID,
 * GKR_ERR_DEVICE. */
int gkr_profile_launches(uint64_t *n, int32_t *cls, int32_t *size_class, float *ms, double *bytes,
                         double *mods);

/* Message for the last error on the calling thread ("" if none). */
const char *gkr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GKR_H */
