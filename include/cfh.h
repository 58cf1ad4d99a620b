/*
 * cfh.h - C ABI of libcfh, the MI355X (gfx950) hot path of the
 * Clifford-fullstate hybrid simulator (CFHS) of arXiv 2602.09020.
 *
 * The simulator state is a pair (F, Phi) (Sec. 4.2, Eq. cfhsstate): F is a
 * Pauli frame (2n Pauli rows effZ_q = U^dag Z_q U, effX_q = U^dag X_q U, the
 * backward interpretation of Sec. 4.1) standing for a Clifford unitary U, and
 * Phi is a 2^n complex amplitude vector; the physical state is U Phi.
 * Clifford gates only update F; a rotation exp(-i theta/2 P) of the physical
 * circuit is applied to Phi as exp(-i theta/2 F(P)) with F(P) = U^dag P U
 * (Eq. single_to_multirot, Eq. Fmap); expectation values are <Phi|F(P)|Phi>
 * (Eq. chfsexp).
 *
 * Conventions used by every call:
 *   - Pauli operators are (x, z, e): P = i^e (x)_j sigma(x_j, z_j) with
 *     sigma(0,0)=I, sigma(1,0)=X, sigma(1,1)=Y, sigma(0,1)=Z (no hidden i in Y),
 *     bit j of x/z = qubit j; in the paper's masks x = m_X|m_Y, z = m_Z|m_Y
 *     (Sec. 2.2).  P is Hermitian iff e is even.
 *   - Qubit j is bit j of an amplitude index; qubit 0 is the least
 *     significant bit (Sec. 3).
 *   - State vectors are device memory, 2^n interleaved (re, im) pairs:
 *     CFH_C128 = two doubles (16 B per amplitude), CFH_C64 = two floats (8 B).
 *     All amplitude arithmetic is done in double precision in registers;
 *     CFH_C64 only changes the storage.
 *   - Rotations are R_P(theta) = exp(-i theta/2 P) (Sec. 3).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued on it and the call returns without waiting,
 *     unless the description says it synchronizes.
 *   - Every call returns a cfh_status; 0 is success.  No C++ exception
 *     crosses this boundary.  On failure cfh_last_error() returns a
 *     thread-local message.
 *   - Host arrays passed in are copied before the call returns; device
 *     pointers passed in stay owned by the caller, who keeps them alive until
 *     the enqueued work has finished.  Handles (frames, plans, Hamiltonians,
 *     batches) are owned by the library and freed by their destroy call.
 *   - Calls may come from several host threads at once.  Calls that use the
 *     same handle or the same device buffers must not overlap in time (the
 *     caller orders them); calls on different handles and buffers are
 *     independent.  The library's own shared state (per-kernel launch
 *     settings, the occupancy cache) is set up under a lock or once; the
 *     allocation-free cfh_expval_noalloc shares one scratch array per GPU
 *     (see there).
 */
#ifndef CFH_H
#define CFH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CFH_API_VERSION 1

typedef int32_t cfh_status;
enum {
    CFH_OK = 0,
    CFH_E_INVAL = -1,         /* null pointer, bad gate code, bad qubit, bad size */
    CFH_E_RANGE = -2,         /* a mask has bits at or above n */
    CFH_E_NOT_HERMITIAN = -3, /* odd phase exponent where a Hermitian operator is required */
    CFH_E_NOMEM = -4,         /* host or device allocation failed */
    CFH_E_HIP = -5,           /* a HIP runtime call failed; message in cfh_last_error() */
    CFH_E_UNSUPPORTED = -6,   /* n or dtype outside what the library supports */
    CFH_E_TIMEOUT = -7        /* a persistent batched run gave up waiting (cfh_batch_results) */
};

typedef enum { CFH_C64 = 0, CFH_C128 = 1 } cfh_dtype;

/* Clifford gate codes (Sec. 2.1 generators H, S, CNOT, plus their common
 * products).  CNOT takes q0 = control, q1 = target.  The one-qubit rotations
 * RX, RY, RZ (exp(-i theta/2 sigma_q), angle given beside the gate) are only
 * for circuits (cfh_circuit_translate / cfh_circuit_run). */
typedef enum {
    CFH_GATE_H = 0, CFH_GATE_S = 1, CFH_GATE_SDG = 2, CFH_GATE_X = 3, CFH_GATE_Y = 4,
    CFH_GATE_Z = 5, CFH_GATE_CNOT = 6, CFH_GATE_CZ = 7, CFH_GATE_SWAP = 8,
    CFH_GATE_RX = 9, CFH_GATE_RY = 10, CFH_GATE_RZ = 11,
    CFH_GATE_MEASURE = 12, /* measure Z_q0 (cfh_circuit_run only; uniform number beside the row) */
    CFH_GATE_RESET = 13    /* prepare |0> on q0: measure Z_q0, then X_q0 on outcome -1 (same) */
} cfh_gate;

/* P = i^e (x)_j sigma(x_j, z_j).  24 bytes, 8-byte aligned. */
typedef struct cfh_pauli {
    uint64_t x;
    uint64_t z;
    int32_t e;        /* phase exponent, taken mod 4 */
    int32_t reserved; /* must be 0 */
} cfh_pauli;

/* Planner/kernel parameters.  A zero field means "library default". */
typedef struct cfh_tuning {
    int32_t tile_bits;     /* b: log2 amplitudes per LDS tile (a coset of a b-dim subspace) */
    int32_t low_bits;      /* c: low index bits always inside a tile (coalescing) */
    int32_t max_run;       /* most rotations in one fused pass (<= 32) */
    int32_t lookahead;     /* rotations scanned for commuting reordering; -1 = in order only */
    int32_t unfused;       /* 1 = one HBM pass per rotation (no LDS staging) */
    int32_t block_threads; /* threads per workgroup of the LDS-staged kernel (256) */
    int32_t variant;       /* fused kernel: 0 = default, 1 = LDS-staged (every rotation through LDS),
                              2 = register-tiled (micro-groups of 4 dimensions in registers, LDS
                              only between micro-groups, next coset prefetched into registers;
                              needs tile_bits in 10..13), 3 = register-tiled without the prefetch,
                              4 = register-tiled, one unrolled body per (partner mask, register
                              sign mask, real/imaginary) so member signs cost no instructions,
                              rotations with |sin| <= |cos| in the tangent form (4 FMAs a pair,
                              the product of their cosines applied once per coset),
                              5 = as 4 with the transposes between micro-groups done in two
                              halves through half the LDS (tile_bits 10..14).  Every variant but 1
                              also selects the register-tiled adjoint sweep (1: LDS-staged).
                              Batches: 0 = register-tiled passes on 2^12 tiles for circuits with
                              n >= 12 (LDS-staged for smaller ones), 2 = LDS-staged passes only */
    int32_t batch_items;   /* batched runs: work items per pass (0 = 32); a pass gets more when an item
                              would cover more than 64 tiles */
    int32_t group_mib;     /* batched runs: circuits are scheduled in consecutive groups whose
                              state and lam vectors fit this many MiB (so the 256 MiB Infinity Cache
                              can keep a group resident across its levels); <= 0 = one group */
    int32_t tile_order;    /* register-tiled passes: 0 = cosets that share 128-byte lines (chunks
                              narrower than 128 B) run on the same XCD at the same time, so the line
                              is fetched into one L2 once, and bit-reversed order otherwise;
                              1 = cosets in index order; 2 = bit-reversed coset index (workgroups
                              running together are spread over the whole state) */
    int32_t reg_tile_bits; /* batched runs: log2 amplitudes of the register tiles that circuits with
                              at least that many qubits run on (11..13; 0 = 12) */
} cfh_tuning;

typedef struct cfh_frame_s *cfh_frame;
typedef struct cfh_plan_s *cfh_plan;
typedef struct cfh_ham_s *cfh_ham;
typedef struct cfh_batch_s *cfh_batch;

/* ------------------------------------------------------------------ misc */

/* Library ABI version (CFH_API_VERSION). */
int cfh_version(void);

/* Thread-local message of the last failed call on this thread ("" if none).
 * The pointer stays valid until the next failing call on the same thread. */
const char *cfh_last_error(void);

/* Number of HIP devices visible (0 when none); never fails. */
int cfh_device_count(void);

/* ------------------------------------------------ a1: encode Pauli strings */

/* Letter strings -> (x, z, e) (Sec. 2.2 Pauli masks; Sec. 3 action on basis
 * states).  `letters` is m rows of n bytes, row-major, column j = qubit j,
 * codes 0=I 1=X 2=Y 3=Z.  out[i] gets e = 0 (so Y = sigma(1,1) exactly).
 * Errors: CFH_E_INVAL (null, n outside 1..63, letter > 3). */
cfh_status cfh_pauli_encode(const uint8_t *letters, int n, size_t m, cfh_pauli *out);

/* ------------------------------------------------- a2: Pauli frame tracker */

/* New frame F_origin on n qubits (effZ_q = Z_q, effX_q = X_q; Sec. 2.3,
 * Eq. framemat).  1 <= n <= 63.  *out is owned by the caller until
 * cfh_frame_destroy. */
cfh_status cfh_frame_create(int n, cfh_frame *out);
cfh_status cfh_frame_destroy(cfh_frame f);

/* U <- G U for one Clifford gate G, updating the rows in the backward
 * interpretation (Sec. 4.1): each gate rewrites O(1) rows, each new row a
 * product of at most two old rows, bit-exact in x, z and the sign e.
 * q1 must be -1 for one-qubit gates and a distinct qubit for CNOT/CZ/SWAP.
 * Errors: CFH_E_INVAL (null frame, bad gate code or qubit). */
cfh_status cfh_frame_apply_clifford(cfh_frame f, int gate, int q0, int q1);

/* Same for m gates given as rows (code, q0, q1) of int32, first row first. */
cfh_status cfh_frame_apply_gates(cfh_frame f, const int32_t *gates, size_t m);

/* Copy row q: effZ_q = U^dag Z_q U and effX_q = U^dag X_q U. */
cfh_status cfh_frame_row(cfh_frame f, int q, cfh_pauli *effZ, cfh_pauli *effX);

/* ----------------------------------------------- a3: frame conjugation */

/* out = F(P) = U^dag P U (Eq. Fmap, with the phase of each Y letter taken
 * from effY_j = -i effZ_j effX_j of Eq. framemat), bit-exact.  Any e is
 * accepted and its parity is preserved.  Errors: CFH_E_RANGE (bits >= n). */
cfh_status cfh_frame_conjugate(cfh_frame f, const cfh_pauli *p, cfh_pauli *out);

/* Host loop over m strings; in and out may alias. */
cfh_status cfh_frame_conjugate_many(cfh_frame f, const cfh_pauli *in, cfh_pauli *out, size_t m);

/* Device version (one thread per string, frame rows staged in LDS): in_dev
 * and out_dev are device arrays of m cfh_pauli.  Asynchronous on `stream`.
 * The frame is copied to the device at the call, so later frame updates do
 * not affect already enqueued work. */
cfh_status cfh_frame_conjugate_device(cfh_frame f, const cfh_pauli *in_dev, cfh_pauli *out_dev,
                                      size_t m, void *stream);

/* ------------------------------------------------------ state helpers */

/* psi <- |index> (all zeros except amplitude `index` = 1). */
cfh_status cfh_state_set_basis(void *psi, int n, int dtype, uint64_t index, void *stream);

/* --------------------------------------- a5/a6: one Pauli rotation, one pass */

/* psi <- exp(-i theta/2 P) psi with P = (x, z, e), e in {0, 2} (e = 2 is -P,
 * the sign a frame conjugation can produce).  Amplitude pairs (y, y^x) are
 * updated together (Sec. 3; App. B pair rule):
 *   psi'[y] = cos(theta/2) psi[y] - i sin(theta/2) i^(e - |x&z|) (-1)^|y&z| psi[y^x];
 * x = 0 is the diagonal case (App. B).  One read and one write of the state.
 * Errors: CFH_E_RANGE, CFH_E_NOT_HERMITIAN, CFH_E_UNSUPPORTED (n outside
 * 1..34), CFH_E_INVAL (null psi). */
cfh_status cfh_apply_pauli_rotation(void *psi, int n, int dtype, uint64_t x, uint64_t z, int e,
                                    double theta, void *stream);

/* -------------------------------------------- a4/a7: planned rotation runs */

/* Plan the in-order sequence of m rotations rot[0..m-1] (already conjugated
 * through the frame) on an n-qubit state of the given dtype.  The planner
 * splits the sequence into passes; a pass is a run of rotations whose x
 * masks lie in the span of a b-dimensional subspace V (tile_bits), so that
 * every coset y + V is closed under all of them and is updated in LDS with
 * one HBM read and one write.  Rotations may move earlier only past
 * rotations they commute with (Sec. 2.1, anticommutation flag), which leaves
 * the product unchanged.  `tuning` may be NULL.  Allocates device memory for
 * the plan (not the state).  Errors: CFH_E_RANGE, CFH_E_NOT_HERMITIAN,
 * CFH_E_UNSUPPORTED, CFH_E_NOMEM, CFH_E_HIP. */
cfh_status cfh_plan_create(int n, int dtype, const cfh_pauli *rot, size_t m,
                           const cfh_tuning *tuning, cfh_plan *out);
cfh_status cfh_plan_destroy(cfh_plan p);

/* Host-only planning (no device memory, usable without a GPU): the pass
 * schedule cfh_plan_create would build.  pass_start needs room for m+1
 * entries and order for m; *n_passes receives the pass count P and
 * pass_start[0..P] the prefix offsets into order.  For tools that compare
 * tunings (the autotuner's cost model) and for tests of the planner. */
cfh_status cfh_plan_dry_run(int n, int dtype, const cfh_pauli *rot, size_t m, const cfh_tuning *tuning,
                            int64_t *n_passes, int64_t *pass_start, int64_t *order);

/* Plan summary: passes, rotations, tile bits actually used, the number of
 * HBM bytes one application moves (2 * 2^n * bytes per amplitude per pass)
 * and the fused kernel variant the plan runs (as in cfh_tuning.variant after
 * resolving the default; 0 for an unfused plan).  Any pointer may be NULL. */
cfh_status cfh_plan_info(cfh_plan p, int64_t *n_passes, int64_t *n_rot, int32_t *tile_bits,
                         double *hbm_bytes, int32_t *variant);

/* Pass boundaries and order: pass_start has n_passes+1 entries (prefix
 * offsets into order), order has m rotation indices in application order. */
cfh_status cfh_plan_schedule(cfh_plan p, int64_t *pass_start, int64_t *order);

/* Coverage of the compile-time rotation bodies (for tests): counts[512]
 * gets, for each body of the register-tiled pass kernel, how many rotations
 * of the plan's passes (inverse = 0: forward order, 1: the inverse sweep)
 * run it with the angles theta_host (host, m entries).  Body index =
 * cx | zr << 4 | tangent << 8: the partner mask and the register sign mask
 * in register coordinates (they also fix whether the pair coefficient is
 * imaginary), and the tangent form (taken when |sin(theta/2)| <=
 * |cos(theta/2)| and the plan's kernel has it).  Host only.  Errors:
 * CFH_E_INVAL (null), CFH_E_UNSUPPORTED (an unfused or LDS-staged plan). */
cfh_status cfh_plan_leaf_counts(cfh_plan p, const double *theta_host, int inverse, int64_t *counts);

/* psi <- R_{m-1} ... R_0 psi with R_k = exp(-i theta_dev[k]/2 rot[k])
 * (inverse = 0), or the inverse product R_0^dag ... R_{m-1}^dag psi
 * (inverse = 1).  theta_dev: device array of m doubles.  Allocates nothing
 * and never synchronizes; uses plan-owned scratch, so calls on one plan must
 * not overlap in time. */
cfh_status cfh_apply_plan(cfh_plan p, void *psi, const double *theta_dev, int inverse,
                          void *stream);

/* ----------------------------------------- a8: Hamiltonian expectation value */

/* Prepare H = sum_j coeff[j] terms[j] (terms already conjugated through the
 * frame, e even) for expectation values and H*psi on n-qubit states.  Terms
 * are grouped by x mask.  For <H> the terms are packed into read-only passes
 * of the register-tiled kernel (at most 32 terms per pass on 2^b tiles,
 * b >= 10, by default 11 at complex128 and 12 at complex64; tuning variant 1 or smaller tiles select LDS-staged passes;
 * variant 5 moves the registers between micro-groups in two halves, as
 * 2^14 tiles always do).
 * H*psi runs on register-tiled passes that hold psi and H psi together
 * (the <H> tile capped at 2^13 amplitudes, at least 256 tiles per pass), or
 * on LDS-staged passes where the register-tiled <H> passes are not
 * selected.  Allocates device memory.  Errors as cfh_plan_create. */
cfh_status cfh_ham_create(int n, int dtype, const cfh_pauli *terms, const double *coeff, size_t m,
                          const cfh_tuning *tuning, cfh_ham *out);
cfh_status cfh_ham_destroy(cfh_ham h);

/* Host-only planning (no device memory, usable without a GPU): the
 * register-tiled <H> passes cfh_ham_create would build for these terms
 * (Eq. chfsexp summed pass by pass: each pass reads the state once and adds
 * the terms whose x masks lie in its tile's span).  Arrays are caller-owned:
 * pass_start needs m+1 entries, order and pass_bits m, basis 16*m words.
 * *n_passes receives the pass count P; pass_start[0..P] are prefix offsets
 * into order, which lists term indices in evaluation order; pass p's tile
 * is spanned by the pass_bits[p] index masks basis[16p .. 16p+pass_bits[p]-1]
 * (the rest of its 16 words are zero).  Errors: CFH_E_INVAL (null
 * argument), CFH_E_RANGE and CFH_E_NOT_HERMITIAN (a term), CFH_E_UNSUPPORTED
 * (n outside 1..34, dtype, or a tuning that selects LDS-staged <H> passes). */
cfh_status cfh_ham_dry_run(int n, int dtype, const cfh_pauli *terms, size_t m, const cfh_tuning *tuning,
                           int64_t *n_passes, int64_t *pass_start, int64_t *order, int32_t *pass_bits,
                           uint64_t *basis);
/* Read passes of one <H>, distinct x masks, and the HBM bytes those passes
 * read (2^n * bytes per amplitude each).  Any pointer may be NULL. */
cfh_status cfh_ham_info(cfh_ham h, int64_t *n_passes, int64_t *n_groups, double *hbm_bytes);

/* out_dev[0] + i out_dev[1] = sum_j coeff_j <psi|P_j|psi> (Eq. chfsexp);
 * the imaginary part is 0 up to rounding for Hermitian terms.  out_dev is
 * device memory for 2 doubles.  Deterministic: fixed-order two-stage
 * reduction.  Asynchronous; allocates nothing. */
cfh_status cfh_expval_async(cfh_ham h, const void *psi, double *out_dev, void *stream);

/* Convenience: builds a temporary Hamiltonian, runs cfh_expval_async and
 * synchronizes `stream`; out_host gets 2 doubles (re, im). */
cfh_status cfh_expval(const void *psi, int n, int dtype, const cfh_pauli *terms,
                      const double *coeff, size_t m, double *out_host, void *stream);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * out_dev[0] + i out_dev[1] = sum_j coeff_j <psi|P_j|psi>, as cfh_expval
 * computes it, with nothing allocated, freed or synchronized.  psi is device
 * memory, 2^n amplitudes of dtype (1 <= n <= 34); terms (m Hermitian Paulis,
 * host) and coeff (m doubles, host) are read before the call returns; out_dev
 * is device memory for 2 doubles.  Each term is one read of the state (no
 * fusion).  The per-workgroup partial sums live in a fixed 32 KiB device
 * array of the library (at most 2048 workgroups per launch, so every n up
 * to 34 fits), one copy per device, looked up on the first call on that
 * device; each call overwrites it, so calls that overlap in time on one
 * device race.  Asynchronous on `stream`; deterministic fixed-order
 * reduction.  Errors: CFH_E_INVAL (null state, output, or terms/coeff with
 * m > 0), CFH_E_RANGE, CFH_E_NOT_HERMITIAN, CFH_E_UNSUPPORTED (n, dtype),
 * CFH_E_HIP. */
cfh_status cfh_expval_noalloc(const void *psi, int n, int dtype, const cfh_pauli *terms, const double *coeff,
                              size_t m, double *out_dev, void *stream);

/* out <- H psi (out-of-place; out must not alias psi).  Asynchronous on
 * `stream`; allocates nothing.  Errors: CFH_E_INVAL (null or aliased
 * pointers), CFH_E_HIP. */
cfh_status cfh_ham_apply(cfh_ham h, const void *psi, void *out, void *stream);

/* ------------------------------------------------- a9: adjoint gradient */

/* Adjoint differentiation of E(theta) = <psi|H|psi>, psi = R_{m-1}..R_0 psi_0
 * (the rotations of plan p with angles theta_dev).  On entry psi holds the
 * final state psi_{m} = apply_plan(psi_0); lam is scratch for one state.
 * Computes lam = H psi, then walks the passes backwards: for each rotation k
 * (last first) grad_dev[k] = Im <lam_k| P_k |psi_k> and both vectors are
 * rewound by R_k^dag, in the same LDS pass.  On return psi holds psi_0 again
 * (up to rounding) and grad_dev (device, m doubles) holds dE/dtheta_k.
 * Requires p and h on the same n and dtype.  Asynchronous; allocates
 * nothing. */
cfh_status cfh_adjoint_grad(cfh_plan p, cfh_ham h, void *psi, void *lam, const double *theta_dev,
                            double *grad_dev, void *stream);

/* ----------------------------------- frame flush / amplitude readout */

/* The Clifford rotations R_1..R_m (angles theta_k of pi/2 or pi, each
 * exp(-i theta_k/2 P_k)) that carry the frame back to the identity frame
 * (Sec. 4.3 and the constructive algorithm of App. A): applied to Phi in
 * order they give U Phi, the physical state, up to a global phase.
 * Two rotations per qubit reduce the frame to one-qubit pairs, at most four
 * one-qubit rotations per qubit turn each pair into (Z, X), and the rows are
 * moved to their own qubits by SWAPs written as three commuting pi/2
 * rotations about X_aX_b, Y_aY_b and Z_aZ_b: m <= 9n - 3.  rot and theta are
 * host arrays of cap entries; *m receives the count.  Host only; the frame is
 * not changed.  Errors: CFH_E_INVAL (null argument), CFH_E_RANGE (m > cap,
 * *m set). */
cfh_status cfh_frame_flush_rotations(cfh_frame f, cfh_pauli *rot, double *theta, size_t cap, size_t *m);

/* Flush the frame into the state: psi (device, 2^n amplitudes of dtype, n
 * the frame's) becomes U psi up to a global phase, through a fused plan of
 * the rotations above on `stream`, and the frame becomes the identity, so
 * the amplitudes of psi are the physical ones.  Synchronous (the call waits
 * for the device work); allocates and frees the plan and an angle buffer.
 * Errors: those of cfh_frame_flush_rotations and cfh_plan_create, CFH_E_HIP. */
cfh_status cfh_frame_flush(cfh_frame f, void *psi, int dtype, void *stream);

/* ------------------------------------------- gate-stream circuits */

/* The hybrid dispatch of a compiled circuit (Sec. 4.3, Eq. single_to_multirot):
 * m gate rows (code, q0, q1) of int32 in circuit order, angles[i] the angle
 * of row i when it is RX/RY/RZ (angles may be NULL when there is none).
 * Clifford rows update the frame (cfh_frame_apply_clifford); a rotation of
 * sigma on qubit q becomes the rotation exp(-i theta/2 F(sigma_q)) on Phi,
 * its axis read from the frame as it stands at that point.  The frame ends
 * updated; rot/theta (host, cap entries) receive the rotations on Phi in
 * order and *nrot their count.  Host only.  Errors: CFH_E_INVAL (null
 * argument, bad code or qubit, q1 != -1 on a rotation), CFH_E_RANGE
 * (more rotations than cap, *nrot set, the frame then holds the whole
 * circuit's Cliffords), CFH_E_UNSUPPORTED (a measurement or reset row:
 * those need the state, see cfh_circuit_run). */
cfh_status cfh_circuit_translate(cfh_frame f, const int32_t *gates, const double *angles, size_t m,
                                 cfh_pauli *rot, double *theta, size_t cap, size_t *nrot);

/* Measure the Hermitian Pauli P on psi (device, 2^n amplitudes of dtype):
 * P(+1) = (1 + <P>)/2, the outcome s is +1 when u < P(+1) (u in [0, 1), the
 * caller's uniform random number) and -1 otherwise, and psi collapses to
 * (psi + s P psi) / (2 sqrt(P(s))) in one pass of the pair kernel.  In the
 * hybrid state, measuring sigma_q is measuring F(sigma_q) on Phi (the frame
 * axis, Sec. 4.3 and the gate flow of App. B).  *outcome = s, *prob_plus =
 * P(+1) (may be NULL).  Synchronous (the outcome is read on the host).
 * Errors: CFH_E_INVAL (null, u outside [0, 1)), CFH_E_RANGE,
 * CFH_E_NOT_HERMITIAN, CFH_E_UNSUPPORTED, CFH_E_HIP. */
cfh_status cfh_measure_pauli(void *psi, int n, int dtype, const cfh_pauli *p, double u, int32_t *outcome,
                             double *prob_plus, void *stream);

/* Run the circuit on (frame, psi): psi device, 2^n amplitudes of dtype, n
 * the frame's.  The rows between two measurement or reset rows are
 * translated as above and their rotations applied as one fused plan on
 * `stream`; a MEASURE row on q measures F(Z_q) on psi with angles[i] as its
 * uniform number and writes the outcome (+1/-1) to outcomes[i]; a RESET row
 * does the same and then applies F(X_q) when the outcome was -1.  Afterwards
 * (frame, psi) is the circuit's output state in the hybrid representation
 * (up to a global phase after resets); cfh_frame_flush turns it into
 * physical amplitudes.  tuning as for cfh_plan_create, may be NULL;
 * outcomes (host, m entries) may be NULL when there is no measurement or
 * reset row.  Synchronous; allocates and frees each segment's plan and angle
 * buffer.  Errors: those of cfh_circuit_translate, cfh_plan_create and
 * cfh_measure_pauli, CFH_E_HIP. */
cfh_status cfh_circuit_run(cfh_frame f, const int32_t *gates, const double *angles, size_t m, void *psi, int dtype,
                           const cfh_tuning *tuning, int32_t *outcomes, void *stream);

/* ------------------------------------------------ roofline calibration */

/* Calibration of the HBM roofline (not part of the method): every amplitude
 * of buf (device memory, 2^n amplitudes of dtype, caller-owned scratch;
 * 8 <= n <= 34) is read once, multiplied by a fixed unit phase and written
 * back, one amplitude per thread.  chunk_bits = -1 streams the buffer in index
 * order; chunk_bits = c >= 0 keeps runs of 2^c contiguous amplitudes and
 * bit-reverses the index bits above them, so consecutive runs land far
 * apart (the access pattern of a fused pass whose tile has c contiguous low
 * bits).  nontemporal = 1 uses nontemporal loads and stores.  The HBM bytes
 * are 2 * 2^n * (bytes per amplitude).  Asynchronous on `stream`.
 * Errors: CFH_E_INVAL, CFH_E_UNSUPPORTED, CFH_E_HIP. */
cfh_status cfh_calib_rmw(void *buf, int n, int dtype, int chunk_bits, int nontemporal, void *stream);

/* ----------------------------------------------- a10: batched circuits */

/* One circuit of a batch: n qubits (8..30), its initial basis state, m
 * rotations already conjugated through its frame (e even) with their angles,
 * and its observable of mh terms (conjugated, e even) with coefficients.
 * All arrays are host memory and are copied by cfh_batch_create. */
typedef struct cfh_circuit_desc {
    int32_t n;
    int32_t reserved;
    uint64_t init_index;
    const cfh_pauli *rot;
    const double *theta;
    int64_t m;
    const cfh_pauli *terms;
    const double *coeff;
    int64_t mh;
} cfh_circuit_desc;

/* Build a batch of `count` independent circuits with their own qubit
 * counts, rotations, angles and observables.  By default (tuning variant 0)
 * a circuit with n >= 12 is planned into fused rotation passes on register
 * tiles of 2^12 amplitudes, read-only measurement passes (forward runs),
 * and H psi and adjoint passes on register tiles (gradient runs); smaller
 * circuits, and every circuit under variant 2, use LDS-staged passes on tiles
 * of 2^min(n, tile_bits) amplitudes (default 2^10) only.  Passes are cut
 * into tuning->batch_items work items each (fewer when a pass has fewer
 * tiles; more when an item would cover more than 64 tiles, so that a large
 * circuit's pass spreads over the GPU) and queued level by level across
 * circuits.  Variant 1 plans the same register-tiled passes and runs
 * each run as one persistent kernel (see cfh_batch_run); it needs every
 * circuit to have n >= the register tile and at least one rotation.  States,
 * angles, gradients, partial sums and the work-item tables live in one
 * library-owned device allocation.  tuning may be NULL.
 * Errors: CFH_E_INVAL, CFH_E_RANGE, CFH_E_NOT_HERMITIAN, CFH_E_UNSUPPORTED
 * (n outside 8..30, tile_bits outside 8..11 for c128 or 8..12 for c64,
 * reg_tile_bits outside 11..13, variant outside 0..2, a variant-1 circuit
 * below the register tile), CFH_E_NOMEM, CFH_E_HIP. */
cfh_status cfh_batch_create(const cfh_circuit_desc *circ, int count, int dtype, const cfh_tuning *tuning,
                            cfh_batch *out);
cfh_status cfh_batch_destroy(cfh_batch b);

/* Work items (gradient run), passes, rotations, state bytes, the
 * algorithmic HBM bytes of one forward run and of one gradient run (every
 * pass reads and writes its vectors once), and the number of cache groups
 * the circuits are scheduled in.  Any pointer may be NULL. */
cfh_status cfh_batch_info(cfh_batch b, int64_t *n_items_grad, int64_t *n_passes, int64_t *n_rot,
                          double *state_bytes, double *bytes_fwd, double *bytes_grad, int32_t *n_groups);

/* Replace all angles (host array, concatenated in circuit order); synchronous. */
cfh_status cfh_batch_set_theta(cfh_batch b, const double *theta_host);

/* Run every circuit: build its initial state, apply its rotations, reduce
 * its energy E_i = <psi_i|H_i|psi_i> (Eq. chfsexp) and, with with_grad = 1,
 * its adjoint gradient dE_i/dtheta.  Every circuit is a chain of passes;
 * level l holds pass l of every circuit whose chain is that long.  The call
 * enqueues on `stream`, in order: a kernel that clears the per-circuit
 * timestamps, a kernel that turns the angles into (cos, sin) tables, then
 * for each level one launch per kernel kind that has items at that level
 * (register-tiled forward, measurement, H psi and adjoint passes; LDS-staged
 * passes), followed by one launch that reduces the level's per-item partial
 * sums in a fixed order.  Kernel boundaries order the levels: no workgroup
 * waits for another, and there is no device queue and no time-out.
 * Asynchronous; allocates nothing and calls no memset, so it can be captured
 * in a hipGraph (cfh_batch_graph_launch).  Runs on one batch must not overlap
 * in time, since they share its device buffers.
 *
 * A variant-1 batch enqueues two kernels instead: one that clears the run's
 * per-pass counters, control words and timestamps and computes the
 * (cos, sin) table, then one persistent kernel on the workgroups the device
 * keeps resident.  Its workgroups take work items from one device counter in
 * a fixed claim order in which every item follows all items of the pass
 * before it in its circuit's chain; a workgroup waits (agent-scope acquire)
 * until that pass is marked ready, runs the item, publishes its stores
 * (agent-scope release) and counts it; the workgroup that finishes a pass
 * reduces its partial sums in the same fixed order as the level launches
 * and marks it ready.  Energies and gradients are therefore bitwise equal to
 * those of variant 0 with the same tuning.  Since items are claimed in that
 * order and only by running workgroups, the run completes whatever number
 * of workgroups is resident.  Each wait is bounded (2 s of device wall clock
 * by default, cfh_batch_persist_config); a workgroup whose wait runs out
 * raises an abort word that makes every workgroup leave, so the kernel always
 * ends, and cfh_batch_results then reports CFH_E_TIMEOUT.
 *
 * Errors: CFH_E_INVAL (null batch), CFH_E_UNSUPPORTED (a tile size the
 * kernels were not built for), CFH_E_HIP (a launch failed; the message is in
 * cfh_last_error). */
cfh_status cfh_batch_run(cfh_batch b, int with_grad, void *stream);

/* Variant-1 batches: a dependency wait gives up after max_wait_s seconds
 * (0 < max_wait_s <= 600) of device wall clock; hold = 1 makes every wait
 * need a ready value that is never written, so every run gives up (the
 * give-up path, for tests); max_grid > 0 runs the persistent kernel on that
 * many workgroups, which completes whether or not they fit on the device at
 * once (0: as many as the occupancy calculation says fit).  Drops captured graphs,
 * which hold the old kernel arguments.  Applies from the next run.
 * Errors: CFH_E_INVAL, CFH_E_UNSUPPORTED (not a variant-1 batch). */
cfh_status cfh_batch_persist_config(cfh_batch b, double max_wait_s, int hold, int max_grid);

/* Variant-1 batches: the grid of the last persistent launch (0 before the
 * first) and the tickets (work items) of a forward and of a gradient run.
 * Any pointer may be NULL.  Errors: CFH_E_INVAL, CFH_E_UNSUPPORTED. */
cfh_status cfh_batch_persist_info(cfh_batch b, int32_t *grid, int64_t *tickets_fwd, int64_t *tickets_grad);

/* The claim order that variant-1 runs use, on the host only (no device):
 * `count` chains of chain_len[c] passes, numbered consecutively chain after
 * chain; pass p has pass_items[p] >= 1 work items; circ_amps[c] weights a
 * circuit's passes (2^n).  Writes ticket_pass / ticket_item (sum of
 * pass_items entries each) and prev (one per pass: the pass before it in its
 * chain, -1 for a chain's first pass).  Level by level; within a level the
 * circuits with the most work left (amps x passes left) come first.
 * Errors: CFH_E_INVAL (null or negative sizes, a pass without items). */
cfh_status cfh_batch_order(int count, const int32_t *chain_len, const int32_t *pass_items,
                           const double *circ_amps, int32_t *ticket_pass, int32_t *ticket_item,
                           int32_t *prev);

/* Capture cfh_batch_run(b, with_grad) into a hipGraph on the first call for
 * that with_grad value, then launch the instantiated graph.  `stream` must
 * be a created (non-default) stream, since the default stream cannot be
 * captured. */
cfh_status cfh_batch_graph_launch(cfh_batch b, int with_grad, void *stream);

/* Synchronize `stream`, then copy results to host: energies[count], grads
 * (concatenated per circuit, sum of m), per-circuit device wall-clock stamps
 * t_start[count] / t_end[count] and the clock rate in Hz.  Any output
 * pointer may be NULL.  Errors: CFH_E_INVAL, CFH_E_HIP, CFH_E_TIMEOUT (a
 * variant-1 run gave up waiting; the copied results are incomplete). */
cfh_status cfh_batch_results(cfh_batch b, double *energies, double *grads, uint64_t *t_start,
                             uint64_t *t_end, double *tick_hz, void *stream);

/* Copy circuit i's current state (2^n_i amplitudes of the batch dtype) to
 * device memory dst_dev, asynchronously on `stream`.  After a gradient run
 * the states have been rewound to the initial states. */
cfh_status cfh_batch_state(cfh_batch b, int i, void *dst_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CFH_H */
