// launch_args.hpp -- kernel argument blocks and the pure-frame schedule.
#pragma once

#include <cstdint>
#include <vector>

#include "device_program.hpp"

namespace symft {

struct Program;

// Aggregate-count mode (detector postselection and the per-shot discarded /
// logical-error flags of the paper's Sec. 6): no record rows are written; a
// shot is discarded when any postselected detector fires, and a kept shot has
// a logical error when any observable differs from its expected value.
struct CountArgs {
    const uint32_t *post;         // bit d: detector d is postselected
    const uint32_t *obs_exp;      // bit o: expected value of observable o
    const uint32_t *chk_off;      // active kernel: n_instr + 1 offsets into chk_mo
    const uint32_t *chk_mo;       // per postselected detector whose last record instruction i makes: the
                                  // offset of its measurement ids in chk_meas (one more entry at the end)
    const uint32_t *chk_meas;
    uint64_t *flags;              // [2][n_words] (row 0 discarded, row 1 logical error) or nullptr
    unsigned long long *counts;   // [2] discarded shots, kept shots with a logical error (added to), or nullptr
    uint32_t on, pad;
};

struct ActiveArgs {
    DevProg P;
    uint64_t seed;
    uint64_t word_begin;      // global index of the first word of the call
    uint64_t n_words;
    uint64_t shots;           // shots of the call (masks the last word)
    uint64_t *out;            // records, record-major
    uint64_t row_stride;
    uint32_t sections;        // bit0 records, bit1 detectors, bit2 observables
    uint32_t tps;             // threads per shot group
    void *scratch;            // HBM vectors (nullptr when LDS-resident)
    uint64_t scratch_stride;  // elements per group slice
    double *p0_out;           // probe: [shot][n_meas] or nullptr
    double *amp_out;          // probe: final active vector [shot][2^amp_k] as (re, im) FP64 pairs, or nullptr
    uint64_t probe_shot0, probe_n;
    uint32_t amp_k;
    uint32_t part_log2;       // count mode: each word split into 2^part_log2 work units of consecutive shots
    uint32_t lds_vec;         // 1: vectors in LDS
    uint32_t lds_bytes;
    uint32_t *unit_counter;   // count mode: workgroups take units from this counter (zeroed before the
                              // launch); nullptr: workgroup b takes units b, b + grid, ...
    CountArgs cnt;
};

// One item of the batched work queue: words [w0, w1) of call `call`.
struct BatchItem {
    uint32_t call, pad;
    uint64_t w0, w1;
};

struct BatchArgs {
    const ActiveArgs *calls;   // device array, one per program of the batch
    const BatchItem *items;    // device array, decreasing estimated cost
    uint32_t *counter;         // next item (reset by a one-thread kernel before each launch)
    uint32_t n_items, pad;
};

struct FrameArgs {
    DevProg P;
    uint64_t seed;
    uint64_t word_begin;
    uint64_t n_words;
    uint64_t shots;
    uint64_t *out;
    uint64_t row_stride;
    uint64_t *scratch;        // per workgroup: flip entries [TW words][sum of class capacities], fallback walk positions
    uint32_t word_entries;    // sum of class capacities (flip entries per word)
    uint32_t cap_override;    // nonzero: every class keeps this many entries (offsets c * cap_override)
    uint32_t sections;
    uint32_t store16;         // output rows may be stored 16 bytes at a time
    uint32_t lds_bytes;
    uint32_t pad;
    CountArgs cnt;
};

struct WaveArgs {
    DevProg P;
    uint64_t seed;
    uint64_t word_begin;
    uint64_t n_words;
    uint64_t shots;
    uint64_t *out;
    uint64_t row_stride;
    uint32_t *scratch;        // per workgroup: slot flip entries [16 words][word_entries]
    uint32_t word_entries;    // sum of class capacities
    uint32_t cap_override;    // nonzero: every class keeps this many slot flips (offsets c * cap_override)
    uint32_t sections;
    uint32_t store16;
    uint32_t lds_bytes;
    uint32_t pad;
    CountArgs cnt;
};

// Pure-frame schedule (programs with peak active width 0); steps run in
// order, separated by workgroup barriers.  Each step is FR_STEP_WORDS words:
//   [kind, a, b, c, 0, next EMIT first node, next EMIT node count, next NOISE class]
//   NOISE  a = class, b = rank end, c = step index within the class: apply the
//          noise events of those channels of the class by XOR-ing each
//          event's lane bit into the slots of its consumers;
//   EMIT   a = first node, b = node count <= FR_LEVEL_MAX: every node of the
//          level reads (and clears) its slot, adds its constant or its
//          RandomMeas word, writes its output row and XORs its value into its
//          successors' slots.
// The "next" fields (node count 0 / class FR_NONE when there is none) let the
// kernel fetch a step's data ahead of the step.
// Node record (8 x uint32): slot | flags << 24 (flags bit0 const, bit1 has
// slot, bit2 RandomMeas, bits 4..5 section: 1 record, 2 detector,
// 3 observable, 0 hidden), output row, the measurement whose RandomMeas word
// is added, push count, first two successor slots, offset of further
// successors in the push list, 0.
enum FrameStepKind : uint32_t { FR_NOISE = 1, FR_EMIT = 2 };
static const uint32_t FR_NO_ROW = 0xFFFFFFFFu;
static const uint32_t FR_LEVEL_MAX = 256;  // nodes per EMIT step: two (node, 4 words) tasks per thread
static const uint32_t FR_STEP_WORDS = 8;
static const uint32_t FR_NONE = 0xFFFFFFFFu;

// Wave-owned schedule (sample_frame_wave.hip): each wave of a 16-wave
// workgroup owns one 64-shot word of a 16-word tile for the whole schedule,
// so nothing but the row staging is shared between waves.  The schedule is a
// list of ops of WV_OP_WORDS words:
//   WV_NOISE  [kind, class, rank end, step index within the class, class of the next NOISE op]
//             XOR the lane bits of the word's flip entries of that step into its slots;
//   WV_BATCH  [kind, first node, node count <= 64, staging position, staging buffer,
//              first node of the next BATCH op, its node count]
//             one node per lane: read and clear the node's slot, add its constant or
//             RandomMeas word, stage the value, XOR it into the successors' slots;
//             no node of a batch depends on another node of the same batch;
//   WV_FLUSH  [kind, offset into the staged-row table, staged rows, staging buffer]
//             workgroup barrier, then the 16 waves store the staged rows as whole
//             128-byte lines (buffers alternate, so staging goes on during the stores).
enum WaveOpKind : uint32_t { WV_NOISE = 1, WV_BATCH = 2, WV_FLUSH = 3 };
static const uint32_t WV_OP_WORDS = 8;
static const uint32_t WV_BATCH_MAX = 64;   // nodes per batch: one per lane
static const uint32_t WV_STAGE_ROWS = 128; // staged rows per buffer: (row, 2 words) per thread of 16 waves
static const uint32_t WV_TILE = 16;        // words per tile = waves per workgroup

struct FrameSchedule {
    std::vector<uint32_t> steps;      // FR_STEP_WORDS per step
    std::vector<uint32_t> first_emit = {0, 0};  // first EMIT step: first node, node count
    uint32_t first_noise_cls = 0xFFFFFFFFu;     // class of the first NOISE step
    std::vector<uint32_t> nodes;    // 8 per node
    std::vector<uint32_t> push;
    std::vector<uint32_t> nodes16;  // 4 per node, the step-synchronous kernel's compact records
    std::vector<uint32_t> push16;   // their lists: a RandomMeas node's measurement, then successor slots
    std::vector<uint64_t> chinfo;   // indexed by class offset + rank
    std::vector<uint64_t> frec;     // per (channel, branch): 16-byte flip record, two entries (see pack_record)
    std::vector<uint64_t> fl3;      // flip entries past a record's two: (k - 1) << 6 | four 12-bit slots
    bool rec_ok = false;            // slots below 2^12 (the step kernel's entries)
    std::vector<uint32_t> cls_cap;  // flip entries kept per (word, class)
    std::vector<uint32_t> ci32;     // per (class, rank): flip-table offset | J << 20 (uniform channels)
    std::vector<uint8_t> st8;       // per (class, rank): NOISE step index within the class
    bool ltab_ok = false;           // every channel uniform, flip-table offsets below 2^20
    uint32_t n_slots = 0;
    size_t n_steps = 0;
    uint32_t max_level = 0;
    uint64_t n_pushes = 0;
    uint64_t n_flips = 0;           // slot flips over all (channel, branch) entries
    double events_per_word = 0;     // expected noise events of one 64-shot word
    bool ok = false;                // the pure-frame kernel can run the program
    // wave-owned schedule
    std::vector<uint32_t> wops;     // WV_OP_WORDS per op
    std::vector<uint32_t> wrows;    // output row of every staged position, by FLUSH offset
    std::vector<uint64_t> wfl;      // per (channel, branch), indexed like fltab: n (1..3) | slots at bits 16, 32, 48;
                                    // or 0 | count << 8 | offset into wsl << 32 (count 0: no flips)
    std::vector<uint16_t> wsl;      // slot lists of the branches that flip more than three
    std::vector<uint32_t> rm_meas;  // measurement of each RandomMeas node, in node order (node word 7 = index)
    std::vector<uint32_t> wcap;     // per class: slot flips kept per word
    uint32_t w_first_noise_cls = 0xFFFFFFFFu;
    uint32_t w_first_batch[2] = {0, 0};
    uint64_t w_n_batches = 0, w_n_flushes = 0;
    bool wave_ok = false;           // the wave-owned schedule was built
};

void build_frame_schedule(const Program &P, FrameSchedule &F);

}  // namespace symft
