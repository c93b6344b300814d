// frame_schedule.cpp -- lowering of a pure-frame program (peak active width 0)
// to the push-based schedule run by the frame kernel.
//
// Every record is an affine function of noise symbols, RandomMeas bits and
// earlier records (paper Sec. 5: DetMeas assigns lambda ^ eta; RandomMeas is
// uniform).  Walking the circuit in order, consecutive noise channels become
// NOISE steps (one per probability class, a contiguous rank range) and
// consecutive measurement / detector nodes become EMIT levels, split where a
// node depends on another node of the same level.  A node with any incoming
// contribution (a noise symbol of its sign, or an earlier record it XORs in)
// owns an accumulator slot from the step of its first contribution to the
// step that emits it; slots are interval-coloured, and a slot is reused only
// by an interval that starts strictly after the previous one ended.
#include <algorithm>
#include <cmath>
#include <map>
#include <queue>

#include "launch_args.hpp"
#include "program.hpp"

namespace symft {

// A flip-table entry: count in bits 0..7; up to two slots inline in bits
// 8..35 and 36..63, otherwise bits 8..35 index the slot list (count 255 means
// the list starts with its own length).
static uint64_t pack_flips(const std::vector<uint32_t> &fl, std::vector<uint32_t> &store) {
    const uint64_t n = fl.size();
    if (n <= 2) {
        uint64_t e = n;
        if (n > 0) e |= (uint64_t)fl[0] << 8;
        if (n > 1) e |= (uint64_t)fl[1] << 36;
        return e;
    }
    const uint64_t off = store.size();
    if (n >= 255) store.push_back((uint32_t)n);
    store.insert(store.end(), fl.begin(), fl.end());
    return (n >= 255 ? 255 : n) | (off << 8);
}

void build_frame_schedule(const Program &P, FrameSchedule &F) {
    F = FrameSchedule();
    if (P.k_max != 0) return;
    uint64_t fl_total = 0;
    for (const Channel &ch : P.chans) fl_total += ch.J;
    if (fl_total >= (1u << 26)) return;  // event records hold 26-bit flip-table indices
    for (const NoiseClass &nc : P.classes)
        if (nc.chans.size() > (1u << 25)) return;  // class stream positions are 32-bit
    const uint32_t M = (uint32_t)P.n_meas, D = (uint32_t)P.n_det, B = (uint32_t)P.n_obs;
    const uint32_t NN = M + D + B;
    struct Node {
        uint8_t cst = 0, rm = 0, sec = 0;
        uint32_t row = FR_NO_ROW, meas = 0;
        std::vector<uint32_t> preds, succs, noise;
        int emit = -1, first = 1 << 30, slot = -1;
    };
    std::vector<Node> nd(NN);
    for (uint32_t t = 0; t < M; ++t) {
        const Instr &I = P.instrs[(size_t)P.meas_instr[t]];
        Node &v = nd[t];
        v.meas = t;
        if (I.kind == RANDOM_MEAS) {
            v.rm = 1;
        } else {
            v.cst = (uint8_t)(I.lam.c ^ I.eta);
            v.preds = I.lam.meas;
            v.noise = I.lam.noise;
        }
        if (P.meas_row[t] >= 0) {
            v.row = (uint32_t)P.meas_row[t];
            v.sec = 1;
        }
    }
    for (uint32_t d = 0; d < D; ++d) {
        Node &v = nd[M + d];
        v.preds = P.det_meas[d];
        v.row = (uint32_t)(P.n_rec + d);
        v.sec = 2;
    }
    for (uint32_t b = 0; b < B; ++b) {
        std::map<uint32_t, int> par;
        for (uint32_t t : P.obs_meas[b]) par[t] ^= 1;
        Node &v = nd[M + D + b];
        for (auto &kv : par)
            if (kv.second) v.preds.push_back(kv.first);
        v.row = (uint32_t)(P.n_rec + P.n_det + b);
        v.sec = 3;
    }
    for (uint32_t i = 0; i < NN; ++i)
        for (uint32_t u : nd[i].preds) nd[u].succs.push_back(i);

    // items in circuit order: (op, kind, id); kind 0 channel, 1 measurement, 2 detector
    struct Item {
        int64_t op;
        int kind;
        uint32_t id;
    };
    std::vector<Item> items;
    for (uint32_t c = 0; c < P.chans.size(); ++c)
        if (P.chans[c].cls >= 0) items.push_back({P.chans[c].op, 0, c});
    for (uint32_t t = 0; t < M; ++t) items.push_back({P.instrs[(size_t)P.meas_instr[t]].op, 1, t});
    for (uint32_t d = 0; d < D; ++d) items.push_back({P.det_op[d], 2, M + d});
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
        if (a.op != b.op) return a.op < b.op;
        return a.kind < b.kind;
    });
    for (uint32_t b = 0; b < B; ++b) items.push_back({(int64_t)P.n_ops, 3, M + D + b});

    // steps
    struct Step {
        uint32_t kind;
        uint32_t cls, r0, r1;
        std::vector<uint32_t> nodes;
    };
    std::vector<Step> steps;
    std::vector<int> chan_step(P.chans.size(), -1);
    std::map<uint32_t, std::pair<uint32_t, uint32_t>> seg;  // class -> rank range
    std::vector<uint32_t> seg_chans;
    std::vector<uint32_t> level;
    std::vector<uint8_t> in_level(NN, 0);
    auto flush_noise = [&]() {
        for (auto &kv : seg) {
            Step s;
            s.kind = FR_NOISE;
            s.cls = kv.first;
            s.r0 = kv.second.first;
            s.r1 = kv.second.second;
            steps.push_back(s);
            for (uint32_t c : seg_chans)
                if ((uint32_t)P.chans[c].cls == kv.first) chan_step[c] = (int)steps.size() - 1;
        }
        seg.clear();
        seg_chans.clear();
    };
    auto flush_level = [&]() {
        if (level.empty()) return;
        Step s;
        s.kind = FR_EMIT;
        s.cls = s.r0 = s.r1 = 0;
        s.nodes = level;
        steps.push_back(s);
        for (uint32_t v : level) {
            nd[v].emit = (int)steps.size() - 1;
            in_level[v] = 0;
        }
        F.max_level = std::max<uint32_t>(F.max_level, (uint32_t)level.size());
        level.clear();
    };
    for (const Item &it : items) {
        if (it.kind == 0) {
            flush_level();
            const Channel &ch = P.chans[it.id];
            auto f = seg.find((uint32_t)ch.cls);
            if (f == seg.end()) seg[(uint32_t)ch.cls] = {(uint32_t)ch.rank, (uint32_t)ch.rank + 1};
            else f->second.second = (uint32_t)ch.rank + 1;
            seg_chans.push_back(it.id);
        } else {
            flush_noise();
            bool dep = false;
            for (uint32_t u : nd[it.id].preds) dep |= in_level[u] != 0;
            if (dep) flush_level();
            level.push_back(it.id);
            in_level[it.id] = 1;
        }
    }
    flush_noise();
    flush_level();

    // noise symbol -> channel
    std::vector<int32_t> sym_chan(P.n_noise_sym, -1);
    for (uint32_t c = 0; c < P.chans.size(); ++c)
        for (uint32_t s = 0; s < P.chans[c].nsym; ++s) sym_chan[P.chans[c].sym0 + s] = (int32_t)c;
    // first contribution of each node
    for (uint32_t i = 0; i < NN; ++i) {
        Node &v = nd[i];
        for (uint32_t s : v.noise) {
            int32_t c = sym_chan[s];
            if (c >= 0 && chan_step[(size_t)c] >= 0) v.first = std::min(v.first, chan_step[(size_t)c]);
        }
        for (uint32_t u : v.preds) v.first = std::min(v.first, nd[u].emit);
    }
    // interval colouring
    std::vector<uint32_t> order;
    for (uint32_t i = 0; i < NN; ++i)
        if (nd[i].first < (1 << 30)) order.push_back(i);
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return nd[a].first < nd[b].first; });
    std::priority_queue<std::pair<int, uint32_t>, std::vector<std::pair<int, uint32_t>>, std::greater<>> busy;
    std::vector<uint32_t> free_slots;
    uint32_t n_slots = 0;
    for (uint32_t i : order) {
        while (!busy.empty() && busy.top().first < nd[i].first) {
            free_slots.push_back(busy.top().second);
            busy.pop();
        }
        uint32_t s;
        if (!free_slots.empty()) {
            s = free_slots.back();
            free_slots.pop_back();
        } else {
            s = n_slots++;
        }
        nd[i].slot = (int)s;
        busy.push({nd[i].emit, s});
    }
    F.n_slots = n_slots;
    // noise symbol -> consumer slots; (channel, branch) -> slots flipped
    std::vector<std::vector<uint32_t>> cons(P.n_noise_sym);
    for (uint32_t i = 0; i < NN; ++i)
        for (uint32_t s : nd[i].noise) cons[s].push_back((uint32_t)nd[i].slot);
    std::vector<uint64_t> chan_fl(P.chans.size(), 0), chan_thr(P.chans.size(), 0);
    uint64_t thr_off = 0;
    for (size_t c = 0; c < P.chans.size(); ++c) {
        const Channel &ch = P.chans[c];
        chan_thr[c] = thr_off;
        thr_off += ch.thr.size();
        chan_fl[c] = F.fltab.size();
        for (uint32_t j = 0; j < ch.J; ++j) {
            std::map<uint32_t, int> par;
            for (uint32_t i = 0; i < ch.nsym; ++i)
                if ((ch.bmask[j] >> i) & 1u)
                    for (uint32_t sl : cons[ch.sym0 + i]) par[sl] ^= 1;
            std::vector<uint32_t> fl;
            for (auto &kv : par)
                if (kv.second) fl.push_back(kv.first);
            F.n_flips += fl.size();
            F.fltab.push_back(pack_flips(fl, F.flslots));
        }
    }
    for (const NoiseClass &nc : P.classes) {
        for (int32_t c : nc.chans) {
            const Channel &ch = P.chans[(size_t)c];
            F.chinfo.push_back((chan_fl[(size_t)c] & 0xFFFFFFFFull) | ((uint64_t)(ch.J & 0xFF) << 32) |
                               ((uint64_t)ch.uniform << 40) | (chan_thr[(size_t)c] << 41));
        }
        F.events_per_word += (double)nc.chans.size() * 64.0 * std::ldexp((double)nc.p32, -32);
    }
    // encode steps and node records
    std::vector<uint64_t> cls_first(P.classes.size() + 1, 0);
    for (const Step &s : steps) {
        F.steps.push_back((s.kind << 28) | (uint32_t)F.data.size());
        if (s.kind == FR_NOISE) {
            const NoiseClass &nc = P.classes[s.cls];
            // flip-table index of the first channel past this step (events are kept as flip-table indices)
            const uint64_t bound = s.r1 < nc.chans.size() ? chan_fl[(size_t)nc.chans[s.r1]] : UINT64_C(0xFFFFFFFF);
            F.data.push_back(s.cls);
            F.data.push_back(s.r0);
            F.data.push_back(s.r1);
            F.data.push_back((uint32_t)std::min<uint64_t>(bound, 0xFFFFFFFFull));
            continue;
        }
        F.data.push_back((uint32_t)(F.nodes.size() / 8));
        F.data.push_back((uint32_t)s.nodes.size());
        for (uint32_t id : s.nodes) {
            const Node &v = nd[id];
            uint32_t flags = (v.cst ? 1u : 0u) | (v.slot >= 0 ? 2u : 0u) | (v.rm ? 4u : 0u) | ((uint32_t)v.sec << 4);
            const uint32_t np = (uint32_t)v.succs.size();
            F.nodes.push_back((v.slot >= 0 ? (uint32_t)v.slot : 0u) | (flags << 24));
            F.nodes.push_back(v.row);
            F.nodes.push_back(v.meas);
            F.nodes.push_back(np);
            F.nodes.push_back(np > 0 ? (uint32_t)nd[v.succs[0]].slot : 0u);
            F.nodes.push_back(np > 1 ? (uint32_t)nd[v.succs[1]].slot : 0u);
            F.nodes.push_back((uint32_t)F.push.size());  // pushes beyond the first two
            F.nodes.push_back(0);
            for (uint32_t k = 2; k < np; ++k) F.push.push_back((uint32_t)nd[v.succs[k]].slot);
        }
    }
    F.n_pushes = 0;
    for (uint32_t i = 0; i < NN; ++i) F.n_pushes += nd[i].succs.size();
    F.n_steps = steps.size();
    F.ok = F.n_steps > 0;
}

}  // namespace symft
