// launch_args.hpp -- kernel argument blocks and the pure-frame schedule.
#pragma once

#include <cstdint>
#include <vector>

#include "device_program.hpp"

namespace symft {

struct Program;

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
    uint64_t probe_shot0, probe_n;
    uint32_t lds_vec;         // 1: vectors in LDS
    uint32_t lds_bytes;
};

struct FrameArgs {
    DevProg P;
    uint64_t seed;
    uint64_t word_begin;
    uint64_t n_words;
    uint64_t shots;
    uint64_t *out;
    uint64_t row_stride;
    uint32_t sections;
    uint32_t wpb;             // 64-shot words per workgroup
    uint32_t lds_bytes;
    uint32_t pad;
};

// Pure-frame schedule (programs with peak active width 0).  Steps run in
// order, separated by workgroup barriers:
//   NOISE  data = [class, rank_begin, rank_end]: draw the events of those
//          channels for every word of the tile and XOR each event's symbols
//          into the accumulator slots of the nodes that consume them;
//   EMIT   data = [n, off_0 .. off_{n-1}, node descriptors ...]: every node of
//          the level reads (and clears) its slot, adds its constant or its
//          RandomMeas word, writes its output row and XORs its value into the
//          slots of its successors.
// Node descriptor: [flags, slot, meas, row, n_push, push slots ...] with
// flags bit0 const, bit1 has slot, bit2 RandomMeas, bits 4..5 section
// (1 record, 2 detector, 3 observable, 0 hidden).
enum FrameStepKind : uint32_t { FR_NOISE = 1, FR_EMIT = 2 };
static const uint32_t FR_NO_ROW = 0xFFFFFFFFu;

struct FrameSchedule {
    std::vector<uint32_t> steps;     // (kind << 28) | data offset
    std::vector<uint32_t> data;
    std::vector<uint32_t> sym_off;   // n_sym + 1
    std::vector<uint32_t> sym_slot;  // consumer slots per noise symbol
    uint32_t n_slots = 0;
    size_t n_steps = 0;
    uint32_t max_level = 0;
};

void build_frame_schedule(const Program &P, FrameSchedule &F);
uint32_t frame_words_per_block(const DevProg &P);

}  // namespace symft
