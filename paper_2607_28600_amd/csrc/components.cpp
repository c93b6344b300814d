// components.cpp -- the product-component lowering of a sampling program
// (paper Sec. 6, adaptive product-component representation).
//
// The active coefficient tensor starts as the scalar 1.  A PromoteRot puts a
// new coordinate in the state c|0> - i s'|1>, independent of the others, so
// it starts a component of its own.  A rotation or an active measurement
// couples the coordinates of its masks (X part a, Z part b); when those lie in
// several components, the components are first merged by an exact Kronecker
// product and the instruction then runs on the merged component alone, with
// its masks and pivot renumbered to the component's local coordinates (a
// component's coordinates keep their dense order).  An
// active measurement removes its pivot coordinate from its component.  A
// component is never split again.
//
// All of this depends only on the instruction stream, not on the shot, so it
// is planned once here: per instruction the component (its region in the
// shot's vector buffer and its local width), the merges that run before it,
// and a region for every component such that regions of components alive at
// the same time do not overlap.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "program.hpp"

namespace symft {

namespace {

struct Comp {
    uint32_t w = 0;     // current width
    uint32_t cap = 0;   // width at birth: the largest it has (widths only shrink after birth)
    int64_t born = 0;   // event index of its creation
    int64_t last = 0;   // event index of its last use
    uint32_t off = 0;   // region offset (amplitudes)
};

// Per-amplitude flops of a dense instruction at the width before it (the
// same weights as the program's dense-flop count).
double flops_of(uint8_t kind, double N) {
    switch (kind) {
    case PROMOTE_ROT: return 4 * N;
    case ACTIVE_DIAG_ROT: return 6 * N;
    case ACTIVE_PAIR_ROT: return 6 * N;
    case ACTIVE_DIAG_MEAS: return 4 * N + 2 * (N / 2);
    case ACTIVE_PAIR_MEAS: return 8 * N + 6 * (N / 2);
    default: return 0;
    }
}

}  // namespace

void plan_components(const Program &P, ProductPlan &out) {
    out = ProductPlan();
    const size_t n = P.instrs.size();
    out.ins.resize(n);
    std::vector<Comp> comps;
    // dense coordinate -> (component, local coordinate)
    std::vector<std::pair<uint32_t, uint32_t>> slot;
    // merges before each instruction, by component id (offsets filled after allocation)
    struct MergeIds {
        uint32_t dst, src1, src2, m1, w;
    };
    std::vector<std::vector<MergeIds>> merges(n);
    std::vector<uint32_t> comp_of(n, UINT32_MAX);
    for (size_t i = 0; i < n; ++i) {
        const Instr &I = P.instrs[i];
        ProductPlan::PInstr &Q = out.ins[i];
        Q.kind = I.kind;
        const int64_t t_merge = 2 * (int64_t)i, t_instr = 2 * (int64_t)i + 1;
        if (I.kind == RANDOM_MEAS || I.kind == DET_MEAS) continue;
        if (slot.size() != I.k_in) {
            // the dense widths and this bookkeeping disagree: keep the dense stream
            out.valid = false;
            return;
        }
        out.work_dense += flops_of(I.kind, std::ldexp(1.0, I.k_in));
        if (I.kind == PROMOTE_ROT) {
            // the new top coordinate, in a component of its own
            Comp c;
            c.w = c.cap = 1;
            c.born = c.last = t_instr;
            comp_of[i] = (uint32_t)comps.size();
            slot.push_back({(uint32_t)comps.size(), 0u});
            comps.push_back(c);
            Q.kind = PROMOTE_FRESH;
            Q.k_in = 0;
            out.work_product += flops_of(PROMOTE_ROT, 1.0);
            continue;
        }
        // components of the instruction's coordinates, in coordinate order
        const uint32_t sup = I.a | I.b;
        std::vector<uint32_t> L;
        for (uint32_t p = 0; p < 32; ++p)
            if ((sup >> p) & 1u) {
                const uint32_t c = slot[p].first;
                if (std::find(L.begin(), L.end(), c) == L.end()) L.push_back(c);
            }
        while (L.size() > 1) {
            const uint32_t c1 = L[0], c2 = L[1];
            Comp m;
            m.w = m.cap = comps[c1].w + comps[c2].w;
            m.born = m.last = t_merge;
            comps[c1].last = std::max(comps[c1].last, t_merge);
            comps[c2].last = std::max(comps[c2].last, t_merge);
            const uint32_t id = (uint32_t)comps.size();
            // The merged coordinates keep their dense order (local index = rank among the
            // component's dense coordinates), so a pivot that is the highest set bit of a
            // dense mask stays the highest of the local one, and a measurement's compaction
            // reads every source at or above the index it writes.  m1 marks the first
            // component's coordinates among the merged ones.
            uint32_t m1 = 0, r = 0;
            for (auto &s : slot)
                if (s.first == c1 || s.first == c2) {
                    if (s.first == c1) m1 |= 1u << r;
                    s = {id, r++};
                }
            merges[i].push_back({id, c1, c2, m1, m.w});
            comps.push_back(m);
            out.work_product += 4.0 * std::ldexp(1.0, m.w);  // one complex product per amplitude
            L.erase(L.begin(), L.begin() + 2);
            L.insert(L.begin(), id);
        }
        const uint32_t c = L[0];
        comp_of[i] = c;
        comps[c].last = std::max(comps[c].last, t_instr);
        uint32_t al = 0, bl = 0;
        for (uint32_t p = 0; p < 32; ++p) {
            if ((I.a >> p) & 1u) al |= 1u << slot[p].second;
            if ((I.b >> p) & 1u) bl |= 1u << slot[p].second;
        }
        Q.a = al;
        Q.b = bl;
        Q.h = (uint8_t)slot[I.h].second;
        // the kernels' pairings and in-place compactions take the pivot as the highest set bit of
        // the pair mask (a) or, for a diagonal measurement, of b; the dense order inside a
        // component keeps it so
        const uint32_t pm = I.kind == ACTIVE_DIAG_MEAS ? bl : al;
        if (I.kind != ACTIVE_DIAG_ROT && (pm == 0 || 31u - (uint32_t)__builtin_clz(pm) != Q.h)) {
            out.valid = false;
            return;
        }
        Q.k_in = (uint8_t)comps[c].w;
        out.work_product += flops_of(I.kind, std::ldexp(1.0, comps[c].w));
        out.k_local_max = std::max<uint32_t>(out.k_local_max, comps[c].w);
        if (I.kind == ACTIVE_DIAG_MEAS || I.kind == ACTIVE_PAIR_MEAS) {
            // the pivot leaves its component and the dense coordinates above it move down
            const uint32_t hl = slot[I.h].second;
            for (auto &s : slot)
                if (s.first == c && s.second > hl) s.second -= 1;
            slot.erase(slot.begin() + I.h);
            comps[c].w -= 1;
        }
    }
    // Regions: in order of birth, each component takes the lowest offset,
    // aligned to its size, that no component alive at its birth holds.
    std::vector<uint32_t> order(comps.size());
    for (uint32_t j = 0; j < comps.size(); ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return comps[x].born < comps[y].born; });
    std::vector<uint32_t> placed;
    uint64_t top = 0;
    for (uint32_t j : order) {
        Comp &c = comps[j];
        const uint64_t size = (uint64_t)1 << c.cap;
        uint64_t off = 0;
        for (;;) {
            bool clash = false;
            for (uint32_t q : placed) {
                const Comp &o = comps[q];
                if (o.last < c.born) continue;  // dead by then
                const uint64_t os = (uint64_t)1 << o.cap;
                if (off < o.off + os && o.off < off + size) {
                    clash = true;
                    off = ((o.off + os) + size - 1) / size * size;
                    break;
                }
            }
            if (!clash) break;
        }
        c.off = (uint32_t)off;
        top = std::max<uint64_t>(top, off + size);
        placed.push_back(j);
    }
    out.vcap = (uint32_t)std::max<uint64_t>(1, top);
    out.n_comps = (uint32_t)comps.size();
    for (size_t i = 0; i < n; ++i) {
        ProductPlan::PInstr &Q = out.ins[i];
        if (comp_of[i] != UINT32_MAX) Q.base = comps[comp_of[i]].off;
        Q.mg_off = (uint32_t)out.merges.size();
        Q.mg_len = (uint32_t)merges[i].size();
        for (const MergeIds &m : merges[i])
            out.merges.push_back({comps[m.dst].off, comps[m.src1].off, comps[m.src2].off, m.m1, m.w});
    }
    out.n_merges = (uint32_t)out.merges.size();
}

}  // namespace symft
