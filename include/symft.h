/*
 * symft.h -- C ABI of the SymFT per-shot sampling library for AMD Instinct
 * MI355X (gfx950).
 *
 * The library compiles a noisy Clifford-dominated circuit into a SymFT
 * sampling program on the host (symbolic Clifford-Pauli frame factorization,
 * paper Sec. 3, and adaptive stabilizer-coordinate planning, Sec. 4) and
 * replays that program across many shots on the GPU (paper Sec. 5): noise
 * choices and random measurement bits are drawn, affine sign expressions are
 * evaluated by XOR, the dense active-state vector is updated by PromoteRot /
 * ActiveDiagRot / ActivePairRot and sampled by RandomMeas / DetMeas /
 * ActiveDiagMeas / ActivePairMeas, and bit-packed records are written.
 *
 * Conventions (all functions):
 *   - Status codes only; nothing throws across this boundary.  On failure
 *     symft_last_error() returns a thread-local message.
 *   - Pointers marked "host" are read during the call only.  Pointers marked
 *     "device" are HIP device allocations owned by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Sampling calls are asynchronous on that stream.
 *   - Records layout (record-major, bit-packed): row r, word w is
 *     out[r * row_stride_words + w]; bit (s % 64) of word (s / 64) holds
 *     shot s of the call; padding bits of the last word are 0.  Rows are the
 *     visible measurement records in circuit order, then detectors, then
 *     observables.
 *   - Measurement outcome 0 is the +1 eigenvalue (paper Sec. 2).
 *   - Random draws follow a counter-based Philox4x32-10 contract keyed by
 *     (seed, global shot index), so any shot range is reproducible and
 *     shard-independent.
 */
#ifndef SYMFT_H
#define SYMFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t symft_status;
#define SYMFT_OK 0
#define SYMFT_EINVAL (-1)     /* malformed op, null pointer, bad size or offset */
/* Code -2 is reserved for a non-Hermitian Pauli (paper Sec. 2 admits only
 * Hermitian ones) and is never returned: an op names its Pauli by the letters
 * X, Y, Z per qubit and a sign bit `negate`, which can express only the
 * Hermitian operators +-P; a phase of +-i has no encoding.  Letters outside
 * 0..3 are EINVAL. */
#define SYMFT_ENONHERMITIAN (-2)
#define SYMFT_EACAUSAL (-3)   /* a record referenced before it is measured (paper Sec. 5, causality) */
#define SYMFT_EPROB (-4)      /* probability < 0, > 1, or a channel total > 1 (paper Sec. 2) */
#define SYMFT_ECAPACITY (-5)  /* peak active width or scratch need exceeds what the library supports */
#define SYMFT_ENOMEM (-6)     /* host or device allocation failed */
#define SYMFT_EHIP (-7)       /* a HIP runtime call failed */

/* Operation kinds (paper Sec. 2).  Pauli letters: 1 = X, 2 = Y, 3 = Z (0 = I in branches). */
enum symft_op_kind {
    SYMFT_OP_H = 1, SYMFT_OP_S, SYMFT_OP_S_DAG, SYMFT_OP_X, SYMFT_OP_Y, SYMFT_OP_Z, /* 1q Cliffords on each qubit */
    SYMFT_OP_CX, SYMFT_OP_CZ, SYMFT_OP_SWAP,          /* on qubit pairs (q0,q1),(q2,q3),... */
    SYMFT_OP_R,            /* reset each qubit to |0> (unrecorded Z measurement + X feedback); arg must be 0 */
    SYMFT_OP_M,            /* recorded Z measurement of each qubit, reported bit flipped w.p. arg */
    SYMFT_OP_MR,           /* recorded Z measurement, then reset, of each qubit, reported bit flipped w.p. arg */
    SYMFT_OP_X_ERROR,      /* per qubit: X with probability arg */
    SYMFT_OP_DEPOLARIZE1,  /* per qubit: X, Y, Z each with probability arg/3 */
    SYMFT_OP_DEPOLARIZE2,  /* per pair: each of the 15 non-identity two-qubit Paulis with probability arg/15 */
    SYMFT_OP_PAULI_CHANNEL,/* one channel on `qubits` (<= 16): branch j (< 64) applies branch_paulis[j*n..] w.p. probs[j] */
    SYMFT_OP_ROT,          /* R_P(arg) = exp(-i arg P / 2), P = (-1)^negate * prod paulis (paper Sec. 2) */
    SYMFT_OP_MPP,          /* recorded measurement of P = (-1)^negate * prod paulis, reported bit flipped w.p. arg */
    SYMFT_OP_FEEDBACK,     /* apply P if the XOR of records `recs` is 1 */
    SYMFT_OP_DETECTOR,     /* detector row = XOR of records `recs` */
    SYMFT_OP_OBSERVABLE,   /* XOR records `recs` into observable row obs_id */
    SYMFT_OP_TICK          /* ignored */
};

typedef struct {
    uint32_t kind;                 /* enum symft_op_kind */
    uint32_t n;                    /* number of entries in qubits (and paulis) */
    const uint32_t *qubits;        /* host, [n] */
    const uint8_t *paulis;         /* host, [n] letters for ROT / MPP / FEEDBACK; else NULL */
    uint32_t negate;               /* ROT / MPP: sign of P (the Pauli stays Hermitian) */
    double arg;                    /* ROT: theta; X_ERROR / DEPOLARIZE1 / DEPOLARIZE2: p;
                                      M / MR / MPP: readout-flip probability in [0, 1] (see below) */
    uint32_t n_branches;           /* PAULI_CHANNEL */
    const double *probs;           /* host, [n_branches] */
    const uint8_t *branch_paulis;  /* host, [n_branches * n] letters 0..3 */
    uint32_t n_recs;
    const int64_t *recs;           /* host, [n_recs]: absolute record ids, or < 0 = look-back (-1 = last) */
    uint32_t obs_id;               /* OBSERVABLE */
} symft_op;

/* Readout flips (paper Sec. 6, sampling independent symbols: readout flips are
 * exogenous symbols like Pauli noise choices): an M, MR
 * or MPP with arg = p > 0 reports the complement of its outcome with
 * probability p and leaves the post-measurement state that of the true
 * outcome (an MR resets on the true outcome).  Each flip is a one-branch
 * noise channel of probability p placed at its measurement, one per target of
 * M / MR and one for MPP, ranked in circuit order with every other channel.
 * A measurement of P whose flip fires is a measurement of -P: the
 * measurement's own draw (RandomMeas word or uniform) decides the reported
 * bit.  arg = 0 adds no channel.  Errors: EPROB for arg outside [0, 1],
 * EINVAL for a nonzero arg on R. */

typedef struct symft_program symft_program; /* opaque, immutable after compile */

/* Instruction kinds of the sampling program (paper Sec. 5). */
enum symft_instr_kind {
    SYMFT_PROMOTE_ROT = 1, SYMFT_ACTIVE_DIAG_ROT = 2, SYMFT_ACTIVE_PAIR_ROT = 3,
    SYMFT_RANDOM_MEAS = 4, SYMFT_DET_MEAS = 5, SYMFT_ACTIVE_DIAG_MEAS = 6, SYMFT_ACTIVE_PAIR_MEAS = 7
};

typedef struct {
    uint32_t n_qubits;
    uint32_t k_max;                /* peak active width over the program */
    uint64_t n_ops;
    uint64_t n_measurements;       /* all measurements, resets included */
    uint64_t n_records, n_detectors, n_observables, n_rows;
    uint64_t n_instr[8];           /* instruction count by enum symft_instr_kind */
    uint64_t n_channels, n_classes, n_noise_symbols;
    uint64_t expr_noise_nnz;       /* noise-symbol references over all sign expressions */
    uint64_t expr_meas_nnz;        /* measurement-symbol references over all sign expressions */
    double dense_flops_per_shot;   /* algorithmic flops of the dense instructions: per amplitude of the width
                                      before the instruction, PromoteRot 4, ActiveDiagRot 6, ActivePairRot 6,
                                      ActiveDiagMeas 5, ActivePairMeas 11 */
    double dense_bytes_per_shot;   /* one read + one write of the live vector per dense instruction (complex FP32) */
    uint64_t frame_steps;          /* pure-frame schedule: steps (0 when the program needs the active kernel) */
    uint64_t frame_noise_steps;    /* of which noise steps */
    uint64_t frame_slots;          /* live accumulator rows of the schedule */
    uint64_t frame_max_level;      /* largest emit level */
    uint64_t frame_pushes;         /* record-to-consumer XORs over the schedule */
    uint64_t frame_noise_consumers;/* noise-symbol-to-consumer XORs, summed over symbols */
    uint64_t rotations_removed;    /* rotations fused into an earlier one or cancelled (symft_compile_opts) */
    uint64_t frame_kernel;         /* pure-frame kernel of the automatic choice for calls of more than
                                      frame_small_words words: 2 step-synchronous, 1 wave-owned (schedules whose
                                      slots fit only its LDS); 0 when the program runs on the active kernel */
    uint64_t frame_wave_batches;   /* wave-owned schedule: node batches (one node per lane) */
    uint64_t frame_wave_flushes;   /* wave-owned schedule: staged-row flushes (workgroup barriers) */
    uint64_t product_selected;     /* 1: sampling runs the product-component stream (symft_compile_opts) */
    uint64_t product_components;   /* components of that stream: one per PromoteRot and one per merge */
    uint64_t product_merges;       /* Kronecker merges per shot */
    uint64_t product_vector_amplitudes; /* its vector buffer per shot (all component regions) */
    double product_flops_per_shot; /* its algorithmic flops per shot (dense_flops_per_shot's weights on the
                                      components' widths, plus 4 per merged amplitude) */
    uint64_t frame_small_words;    /* pure-frame programs whose automatic kernel is the step-synchronous one:
                                      calls of at most this many 64-shot words take the wave-owned kernel
                                      instead (small schedules, where it is faster); 0 when none do */
} symft_info;

/* Compile options.  simplify = 1 runs a conservative commutation-aware
 * rewrite before planning (paper Sec. 6, simplification before planning):
 * a rotation R_P(b) later in the circuit is fused into an earlier R_P(a) with
 * the same Pauli body (the same qubits and letters; R_-P(t) = R_P(-t)) when
 * every op between them acts on qubits disjoint from P's support and no
 * detector lies between them; the fused rotation is R_P(a + b), and it is
 * removed when a + b is a multiple of 2 pi (global phase dropped).  The
 * fused rotation keeps the earlier rotation's place; the later op becomes a
 * no-op, so per-op arrays keep the circuit's length.  A rotation that reaches
 * a measurement of +-P in the same way (an MPP of the same body; M, MR or R of
 * the qubit when P = Z_q) is removed: before such a measurement R_P is a phase
 * per outcome (the paper's move of a measurement toward a rotation of the same
 * body, which then reduces to a branch phase).  Records, detectors and
 * measurement order are unchanged. */
typedef struct {
    uint32_t simplify;
    uint32_t components;           /* product components (paper Sec. 6): 0 = automatic (used when they at
                                      least halve the dense flops per shot, merges counted, with a vector
                                      buffer no larger than 2^k_max); 1 = never; 2 = always (programs with an
                                      active state whose buffer fits 2^20 amplitudes).  Records are the same
                                      up to the rounding of branch probabilities */
    uint32_t reserved[2];          /* 0 */
} symft_compile_opts;

/* Compile `ops` (paper Sec. 2 circuit) into a sampling program (Sec. 3-4).
 * Host only; no GPU work.  Errors: EINVAL (bad op / qubit / arity), EACAUSAL,
 * EPROB, ECAPACITY (k_max > 30), ENOMEM.  `opts` points to a
 * symft_compile_opts, or is NULL for the defaults (no simplification).
 * On success *out owns the program; free it with symft_program_free. */
symft_status symft_compile(uint32_t n_qubits, const symft_op *ops, size_t n_ops, const void *opts,
                           symft_program **out);

/* Summary counts and the per-shot algorithmic work of the program. */
symft_status symft_program_info(const symft_program *p, symft_info *info);

/* Host introspection of the plan, for tests:
 *   k_after_op[n_ops]     active width after every op;
 *   meas_kind[n_meas]     per measurement 0 random, 1 deterministic, 2 active-diagonal, 3 active-pair;
 *   rot_kind[n_ops]       per op 0 none, 1 promote, 2 active-diagonal, 3 active-pair.
 * Any pointer may be NULL. */
symft_status symft_program_plan(const symft_program *p, int16_t *k_after_op, int8_t *meas_kind, int8_t *rot_kind);

/* Export of the compiled instruction stream, for tests and inspection.
 * Call once with all array pointers NULL to get the counts in *counts
 * (counts[0] instructions, [1] noise refs, [2] measurement refs, [3] channels,
 * [4] branch masks), then again with arrays of those sizes:
 *   instr[n_instr * 13]: kind, k_in, h, mu (power of i), eta, lambda constant,
 *                        a, b, measurement index (-1 none), noise_off,
 *                        noise_len, meas_off, meas_len
 *   theta[n_instr]       rotation angle
 *   noise_refs / meas_refs  symbol lists of each lambda (paper Sec. 3 affine signs)
 *   chan[n_chan * 4]:    first noise symbol, symbol count, branch count,
 *                        offset into bmask
 *   bmask[...]           per branch: bit i set <=> symbol (first + i) is 1 */
symft_status symft_program_export(const symft_program *p, uint64_t *counts, int64_t *instr, double *theta,
                                  uint32_t *noise_refs, uint32_t *meas_refs, int64_t *chan, uint32_t *bmask);

/* Sampling options. */
typedef struct {
    uint64_t shot_offset;          /* global index of the first shot; must be a multiple of 64 */
    uint32_t precision;            /* 0 = complex FP64 amplitudes, 1 = complex FP32 (FP64 scale and threshold) */
    uint32_t sections;             /* bit 0 records, bit 1 detectors, bit 2 observables; 0 means all */
    uint64_t row_stride_words;     /* 0 means ceil(shots / 64) */
    uint32_t frame_entry_cap;      /* pure-frame programs: 0 = automatic; otherwise the number of flip entries
                                      kept per (64-shot word, probability class) before that word falls back to
                                      drawing its events again at every step (records are unchanged; for tests
                                      of that fallback) */
    uint32_t frame_tile_words;     /* pure-frame programs: 0 = automatic (32-word tiles, one 16-wave workgroup
                                      per CU, when the schedule fits LDS at that width and there are at least
                                      two such tiles per CU; else 16-word tiles); 16 or 32 forces the width
                                      (ECAPACITY if it does not fit; records are unchanged) */
    uint32_t frame_kernel;         /* pure-frame programs: 0 = automatic (the step-synchronous kernel when its
                                      LDS fits, else the wave-owned kernel, in which each wave of a 16-wave
                                      workgroup owns one 64-shot word for the whole schedule; the wave-owned
                                      one also for calls of at most symft_info.frame_small_words words);
                                      1 = wave-owned
                                      (ECAPACITY if it does not fit); 2 = step-synchronous.  A nonzero
                                      frame_tile_words selects the step-synchronous kernel.  Records are
                                      unchanged */
    uint32_t active_kernel;        /* programs with an active state: 0 = automatic (symft_autotune's choice,
                                      else the shot-group kernel); 1 = the shot-group kernel (a group of
                                      threads per shot); 2 = the lane kernel (one wave per 64-shot word, one
                                      lane per shot, every shot's vector buffer in LDS; ECAPACITY when that
                                      state passes 64 KB).  Records are the same up to the rounding of branch
                                      probabilities */
} symft_sample_opts;

/* Sample `shots` shots (paper Sec. 5) into device buffer records_out
 * (n_rows x ceil(shots/64) uint64 words, record-major as above), with
 * complex FP64 amplitudes.  shots == 0 is a no-op, and so is a program with
 * no rows (no records, detectors or observables; records_out may then be
 * NULL).  Errors: EINVAL (null program or output), ECAPACITY, ENOMEM, EHIP. */
symft_status symft_sample(const symft_program *p, uint64_t shots, uint64_t seed, uint64_t *records_out,
                          void *stream);

/* As symft_sample with options (shot offset, precision, sections, stride).
 * Rows of sections not requested are left untouched. */
symft_status symft_sample_ex(const symft_program *p, const symft_sample_opts *opts, uint64_t shots, uint64_t seed,
                             uint64_t *records_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): symft_sample_ex
 * with every kernel's scratch taken from a fixed device array of the library
 * (64 MiB per device, held until the process ends) and no allocation by the
 * library.  Arguments, layout and records are those of symft_sample_ex, and
 * the records are identical; to fit the fixed scratch a launch may run fewer
 * workgroups (the pure-frame kernels' flip entries, the active kernel's
 * vector slices when vectors do not fit LDS).
 *   - The program must already be resident on the current device (uploaded
 *     by an earlier symft_sample / symft_sample_ex call there): EINVAL
 *     otherwise.
 *   - ECAPACITY when a single workgroup's scratch exceeds 64 MiB (for
 *     example a peak active width of 23 and above in FP64).
 *   - Every call on one device shares that device's array, which keeps the
 *     last call's contents (nothing in it needs to start at zero: every
 *     region is written before it is read).  Calls that overlap on one device
 *     -- on different streams, or from several threads -- race; serialise
 *     them on one stream. */
symft_status symft_sample_noalloc(const symft_program *p, const symft_sample_opts *opts, uint64_t shots, uint64_t seed,
                                  uint64_t *records_out, void *stream);

/* Sample n programs in one persistent launch (paper Sec. 6 batching across
 * shots, here also across programs): a work queue over (program, word range)
 * items ordered by decreasing cost.  records_out[i] (device, n_rows(i) x
 * ceil(shots[i]/64) words) receives program i's rows for shots[i] shots with
 * seeds[i]; precision as in symft_sample_opts.  Threads per shot follow a
 * rule, not the autotuner: the members share one LDS size (the largest
 * member's), so each member takes the most shot groups per 256-thread
 * workgroup whose vectors fit an LDS budget (at most 64 groups).  The first
 * call with a new argument set builds the plans for budgets of 64 and 32 KB
 * and, when they differ, runs each twice on `stream` (writing the batch's own
 * records, which the call's launch then rewrites) and keeps the faster; that
 * first call synchronises the stream.  `graph` = 1
 * captures the launch (a counter-reset kernel and the persistent kernel) in
 * a HIP graph on first use and replays it on later calls with identical
 * arguments.  Programs that need their own kernel (pure frame, or vectors
 * that do not fit LDS) are sampled by ordinary launches on the same stream.
 * Calls with the same plan must not overlap on the device (they share the
 * queue counter). */
symft_status symft_sample_batch(const symft_program *const *progs, const uint64_t *shots, const uint64_t *seeds,
                                uint64_t *const *records_out, size_t n, uint32_t precision, uint32_t graph,
                                void *stream);

/* Aggregate-count options (paper Sec. 6: detector postselection and the
 * aggregate-count interface). */
typedef struct {
    uint64_t shot_offset;          /* global index of the first shot; must be a multiple of 64 */
    uint32_t precision;            /* as in symft_sample_opts */
    uint32_t n_post;               /* entries in post */
    const uint32_t *post;          /* host, [n_post]: detector indices (0-based, circuit order); a shot in which
                                      any of them is 1 is discarded.  Repeats are allowed.  NULL if n_post = 0 */
    const uint8_t *obs_expected;   /* host, [n_observables] values 0/1, or NULL for all 0: a kept shot has a
                                      logical error when some observable differs from its expected value */
    uint32_t threads_per_shot;     /* programs with a dense active vector: 0 = automatic (the choice of
                                      symft_autotune_counts for this program, postselection set and precision
                                      if it has run; else one shot group per workgroup from peak width 8 on,
                                      so a workgroup leaves a rejected shot at once, and the record path's
                                      choice below); otherwise 4 .. 256, a power of two, or 1024 at peak
                                      width >= 13 (peak widths 13 and 14 run 64 .. 256 with vectors in HBM,
                                      values below 64 as 64; width 15 and above always uses 1024).  From 64
                                      on a workgroup holds one shot group.  1 = the lane kernel (one lane per
                                      shot; a wave leaves the stream once all its shots are discarded;
                                      ECAPACITY when its state passes 64 KB), also a candidate of
                                      symft_autotune_counts.  Flags do not depend on it */
    uint32_t mode;                 /* programs with a dense active vector: 0 = automatic (with threads_per_shot
                                      0, the path symft_autotune_counts timed faster, else 1; with a nonzero
                                      threads_per_shot, 1); 1 = the count kernel, which
                                      stops a rejected shot's dense work; 2 = detector and observable rows
                                      written to scratch by the record kernel, then reduced to the flags (for
                                      programs that reject few shots).  Flags do not depend on it.  Pure-frame
                                      programs always use the frame kernel's flags */
    uint32_t frame_kernel;         /* pure-frame programs, as in symft_sample_opts: 0 automatic, 1 wave-owned,
                                      2 step-synchronous; flags do not depend on it */
} symft_count_opts;

/* Sample `shots` shots and report, per shot, only a discarded flag and a
 * logical-error flag (paper Sec. 6): no record, detector or observable rows
 * are written.
 *   flags_out   device, 2 x ceil(shots/64) uint64 words, or NULL: row 0 bit s
 *               = shot s discarded, row 1 bit s = shot s kept with a logical
 *               error; padding bits are 0.
 *   counts_out  device, 2 uint64, or NULL: the number of discarded shots and
 *               the number of kept shots with a logical error are ADDED to
 *               counts_out[0] and counts_out[1] (so calls over consecutive
 *               shot ranges accumulate; zero it before the first).
 * On programs with a dense active vector a postselected detector is checked
 * right after the instruction that makes its last record, and a rejected
 * shot does no further dense work; with one shot group per workgroup the
 * workgroups take 4-shot units of the words as they free up, so the
 * rejected shots' uneven work balances over the launch.  Flags equal those computed from the full
 * records of symft_sample_ex with the same seed and shot range.
 * Errors: EINVAL (null program, detector index out of range, expected value
 * not 0/1, bad offset), ECAPACITY, ENOMEM, EHIP.  shots == 0 is a no-op. */
symft_status symft_sample_counts(const symft_program *p, const symft_count_opts *opts, uint64_t shots,
                                 uint64_t seed, uint64_t *flags_out, uint64_t *counts_out, void *stream);

/* Autotuner of the aggregate-count mode: times each threads-per-shot
 * configuration (4 .. 256 that fits LDS; at widths 9 .. 12 also 64 .. 256 with
 * vectors in HBM; at peak widths 13 and 14, 64 .. 256 with vectors in HBM and
 * 1024; the lane kernel; rows written by the record kernel, then reduced) on
 * 16384 words of this program up to peak width 8, 4096 at widths 9 .. 12 and 1024 at 13 and 14,
 * with opts' postselection set and precision (opts->threads_per_shot
 * and shot_offset are ignored) and keeps the fastest for later
 * symft_sample_counts calls with the same program, set and precision.
 * Fewer shot groups per workgroup let rejected shots end sooner; more keep
 * the lanes of small vectors busy.  Synchronous; allocates a scratch
 * counter.  *tps_out (nullable) receives the choice (0 for pure-frame
 * programs).  Errors as symft_sample_counts. */
symft_status symft_autotune_counts(const symft_program *p, const symft_count_opts *opts, uint32_t *tps_out);

/* Aggregate counts for n programs in one persistent launch (paper Sec. 6:
 * detector postselection in the batch sampler): symft_sample_counts run
 * inside symft_sample_batch's work queue.  Program i samples shots[i] shots
 * with seeds[i] under opts[i] (host array of n, or NULL: nothing
 * postselected, every observable expected 0); of opts[i] only shot_offset,
 * n_post, post and obs_expected are used (precision is the batch's; the
 * launch configuration is the batch's own).
 *   flags_out   host array of n device pointers, or NULL; an entry is NULL
 *               or 2 x ceil(shots[i]/64) words, as in symft_sample_counts.
 *   counts_out  device, 2n uint64, or NULL: program i's discarded and
 *               logical-error counts are ADDED to counts_out[2i], [2i + 1].
 * A shot group leaves the instruction stream at its rejecting detector, and
 * a work item's groups leave it once all of them are rejected.  Programs
 * that need their own kernel (pure frame, or vectors that do not fit LDS)
 * run as symft_sample_counts calls on the same stream.  `graph`, plan
 * caching and the no-overlap rule as in symft_sample_batch (a replayed graph
 * adds to the counters again).  Errors as symft_sample_counts, plus EINVAL
 * for a NULL program. */
symft_status symft_sample_counts_batch(const symft_program *const *progs, const uint64_t *shots, const uint64_t *seeds,
                                       const symft_count_opts *opts, uint64_t *const *flags_out, uint64_t *counts_out,
                                       size_t n, uint32_t precision, uint32_t graph, void *stream);

/* Autotuner: times each threads-per-shot configuration (4 .. 256) of the
 * active-state kernel that fits LDS on 4096 words of this program (at peak
 * widths 13 and 14: 64 .. 256 with vectors in HBM, and 1024, on 1024 words; at
 * widths 9 .. 12 also 64 .. 256 with vectors in HBM instead of LDS;
 * untuned, those widths run 128 threads per shot in FP32 and 256 in FP64; from
 * width 15 on, 1024 always) and keeps the fastest
 * for the program's (peak active width, precision); later single-program
 * launches with that key use it (batches use their own rule, see
 * symft_sample_batch).  Records do not depend on the
 * choice.  Synchronous; allocates a scratch output.  *tps_out (nullable)
 * receives the choice (0 for pure-frame programs, which have one kernel; 1 for
 * the lane kernel, symft_sample_opts.active_kernel = 2, also a candidate when
 * its state fits). */
symft_status symft_autotune(const symft_program *p, uint32_t precision, uint32_t *tps_out);

/* Probe: Pr(m = 0) of every measurement for shots [shot_begin, shot_begin + n_shots)
 * computed by the same GPU kernels (FP64 or FP32), written to host
 * p0_host[n_shots * n_measurements] (NaN for RandomMeas / DetMeas).
 * Synchronous.  For tests and error reports. */
symft_status symft_probe(const symft_program *p, uint64_t shot_begin, uint32_t n_shots, uint64_t seed,
                         uint32_t precision, double *p0_host);

/* Probe of the final active state: for shots [shot_begin, shot_begin + n_shots)
 * the dense active vector after the last instruction (paper Sec. 4-5: the
 * active amplitudes alpha_x over the 2^k_end active coordinates, k_end the
 * width after the last op as symft_program_plan reports it), computed by the
 * same GPU kernels in FP64 (precision 0) or FP32 (1) and written to host
 * amp_host[n_shots][2^k_end][2] as (re, im) FP64 pairs (nullable: then only
 * *k_end is set).  Pure-frame programs report k_end = 0 and the amplitude
 * 1.  Synchronous.  For tests and FP32 error reports.  Errors: EINVAL,
 * ENOMEM, EHIP. */
symft_status symft_probe_amplitudes(const symft_program *p, uint64_t shot_begin, uint32_t n_shots, uint64_t seed,
                                    uint32_t precision, double *amp_host, uint32_t *k_end);

/* Gap check: the geometric gap G = max { g <= 4096 : v < Q[g] } of the
 * noise draw contract (Q the exact table of a class with per-draw firing
 * probability p32 / 2^32, 0 < p32 <= 2^32) for n draws v (device array),
 * decided exactly as the sampling kernels decide it (table-free margins,
 * else the table), written to device array g_out.  Synchronous.  For tests
 * of the gap decision at table boundaries.  Errors: EINVAL, ENOMEM, EHIP. */
symft_status symft_gap_check(uint64_t p32, const uint32_t *v, int32_t *g_out, uint64_t n, void *stream);

void symft_program_free(symft_program *p);

/* Thread-local message of the last failing call on this thread. */
const char *symft_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SYMFT_H */
