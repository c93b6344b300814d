// program.hpp -- host-side SymFT sampling program produced by symft_compile.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/symft.h"

namespace symft {

enum InstrKind : uint8_t {
    PROMOTE_ROT = 1,
    ACTIVE_DIAG_ROT = 2,
    ACTIVE_PAIR_ROT = 3,
    RANDOM_MEAS = 4,
    DET_MEAS = 5,
    ACTIVE_DIAG_MEAS = 6,
    ACTIVE_PAIR_MEAS = 7,
    // product-component streams only: a PromoteRot whose new coordinate starts a
    // component of its own, written from the amplitude 1 (no source vector)
    PROMOTE_FRESH = 8,
};

// Affine Boolean expression over F2 (paper Sec. 3): constant bit, noise
// symbols and measurement symbols; its value under an assignment is the XOR.
struct Expr {
    uint8_t c = 0;
    std::vector<uint32_t> noise;  // noise symbol ids (0-based)
    std::vector<uint32_t> meas;   // measurement indices
};

struct Instr {
    uint8_t kind = 0;
    uint8_t k_in = 0;   // active width before the instruction
    uint8_t h = 0;      // pivot coordinate (active measurements)
    uint8_t mu = 0;     // mu = i^mu
    uint8_t eta = 0;    // DetMeas / ActiveDiagMeas
    uint32_t a = 0, b = 0;
    double theta = 0;
    int32_t meas = -1;  // measurement index t
    int32_t op = -1;    // source op
    Expr lam;
};

// Noise channel under the draw contract.
struct Channel {
    int32_t op = -1;      // source op
    uint64_t p32 = 0;     // event threshold (<= 2^32)
    int32_t cls = -1;     // probability class, -1 = never fires
    int64_t rank = 0;     // position within the class
    uint8_t uniform = 1;  // branch = (v * J) >> 32
    uint32_t J = 1;       // number of branches
    std::vector<uint64_t> thr;    // non-uniform thresholds
    uint32_t sym0 = 0, nsym = 0;  // noise symbols [sym0, sym0 + nsym)
    std::vector<uint32_t> bmask;  // per branch: bit i <=> symbol sym0 + i is 1
};

// Exact geometric table of the draw contract: Q[0] = 2^32,
// Q[g + 1] = floor(Q[g] (2^32 - p32) / 2^32), g < 4096 (4097 entries).
void gap_table(uint64_t p32, uint64_t *Q);

struct NoiseClass {
    uint64_t p32 = 0;
    std::vector<int32_t> chans;  // channel ids by rank
    std::vector<uint64_t> Q;     // exact geometric table, 4097 entries
};

struct Program {
    uint32_t n_qubits = 0;
    uint32_t k_max = 0;
    uint64_t n_ops = 0, n_meas = 0, n_rec = 0, n_det = 0, n_obs = 0;
    uint32_t n_noise_sym = 0;
    uint64_t rot_removed = 0;  // rotations fused or cancelled by the simplification pass
    std::vector<Instr> instrs;
    std::vector<int32_t> meas_instr;            // measurement -> instruction
    std::vector<int64_t> meas_row;              // measurement -> record row, -1 hidden
    std::vector<std::vector<uint32_t>> det_meas;  // detector -> measurement ids
    std::vector<int32_t> det_op;                  // detector -> source op
    std::vector<std::vector<uint32_t>> obs_meas;  // observable -> measurement ids (XOR, duplicates cancel)
    std::vector<Channel> chans;
    std::vector<NoiseClass> classes;
    // plan introspection
    std::vector<int16_t> k_after_op;
    std::vector<int8_t> meas_kind;
    std::vector<int8_t> rot_kind;
    uint64_t n_rows() const { return n_rec + n_det + n_obs; }
};

// The product-component lowering (paper Sec. 6): per dense instruction, the
// component it runs on (region offset and local width in the shot's vector
// buffer, masks and pivot in local coordinates) and the Kronecker merges that
// run before it.  Index-aligned with Program::instrs.
struct ProductPlan {
    struct PInstr {
        uint8_t kind = 0;   // as the dense instruction, PROMOTE_FRESH for a PromoteRot
        uint8_t k_in = 0;   // local width of the component before the instruction
        uint8_t h = 0;      // local pivot
        uint32_t a = 0, b = 0;
        uint32_t base = 0;  // region offset of the component (amplitudes)
        uint32_t mg_off = 0, mg_len = 0;
    };
    struct Merge {
        uint32_t dst, src1, src2;  // region offsets
        uint32_t m1, w;            // the result's coordinates that come from src1 (bit mask); its width
    };
    std::vector<PInstr> ins;
    std::vector<Merge> merges;
    bool valid = true;         // the plan followed the dense widths (else only the dense stream runs)
    uint32_t vcap = 1;         // amplitudes per shot over all regions
    uint32_t n_comps = 0, n_merges = 0, k_local_max = 0;
    double work_dense = 0;     // algorithmic flops per shot, dense
    double work_product = 0;   // the same for the components, merges included
};
void plan_components(const Program &P, ProductPlan &out);

// Returns 0 or a negative symft status; err receives the message.
int compile_program(uint32_t n_qubits, const void *ops, size_t n_ops, Program &out, std::string &err);

// The conservative commutation-aware rewrite of symft_compile_opts.simplify
// on a validated-shape op list: returns the rewritten list (same length; ops
// it removes become TICK) and the number of rotations removed.  The returned
// ops borrow the input's arrays.
std::vector<symft_op> simplify_rotations(const symft_op *ops, size_t n_ops, uint64_t &removed);

}  // namespace symft
