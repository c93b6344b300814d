// frame_schedule.cpp -- lowering of a pure-frame program (peak active width 0)
// to the push-based schedule run by the frame kernel.
//
// Every record is an affine function of noise symbols, RandomMeas bits and
// earlier records (paper Sec. 5: DetMeas assigns lambda ^ eta; RandomMeas is
// uniform).  Walking the circuit in order, consecutive noise channels become
// NOISE steps (one per probability class, a contiguous rank range) and
// consecutive measurement / detector nodes become EMIT levels.  A node that
// depends on a node of the open level takes that node's expression in place of
// the dependency (values add over GF(2)), so chains of records determined by
// records just made, such as the final data measurements of a memory
// experiment, share one level; a level is split only where that would need
// two RandomMeas words in one node or exceed the size caps.  A node with any incoming
// contribution (a noise symbol of its sign, or an earlier record it XORs in)
// owns an accumulator slot from the step of its first contribution to the
// step that emits it; slots are interval-coloured, and a slot is reused only
// by an interval that starts strictly after the previous one ended.
//
// The slots flipped by each (channel, branch) are pre-packed as flip entries
// of up to three 16-bit slots each (the kernel ORs in the shot lane and the
// step), and every channel carries the index of its NOISE step within its
// class, so a drawn event becomes its entries without further lookups.
#include <algorithm>
#include <cmath>
#include <map>
#include <queue>

#include "launch_args.hpp"
#include "program.hpp"

namespace symft {

// Flip entries of one (channel, branch): ceil(n / 4) entries
// (k - 1) << 6 | s0 << 16 | s1 << 28 | s2 << 40 | s3 << 52 (k = slots in the
// entry, 1..4; slots below 2^12, which every schedule that fits the
// step-synchronous kernel's LDS satisfies).  The branch's 16-byte flip record
// holds the first two entries, the entry count m < 64 in the lane bits
// (0..5) of the first; with m > 2 the others sit in ext from entry 2 X on
// (X even, so a 16-byte load reads two), X stored in the bits that are zero in
// entries at rest: step bits (8..15) of the first entry, lane and step bits of
// the second.  Returns false when a branch has 64 entries or more.
static bool pack_record(const std::vector<uint32_t> &fl, std::vector<uint64_t> &rec, std::vector<uint64_t> &ext) {
    std::vector<uint64_t> es;
    for (size_t i = 0; i < fl.size(); i += 4) {
        const size_t cnt = std::min<size_t>(4, fl.size() - i);
        uint64_t e = (uint64_t)(cnt - 1) << 6;
        for (size_t q = 0; q < cnt; ++q) e |= (uint64_t)(fl[i + q] & 0xFFFu) << (16 + 12 * q);
        es.push_back(e);
    }
    if (es.size() >= 64) return false;
    uint64_t r0 = es.empty() ? 0 : es[0], r1 = es.size() > 1 ? es[1] : 0;
    r0 |= (uint64_t)es.size();
    if (es.size() > 2) {
        const uint64_t x = ext.size() / 2;  // in 16-byte units
        if (x >= (1u << 22)) return false;
        ext.insert(ext.end(), es.begin() + 2, es.end());
        if (ext.size() & 1) ext.push_back(0);
        r0 |= (x & 0xFFu) << 8;
        r1 |= ((x >> 8) & 63u) | (((x >> 14) & 0xFFu) << 8);
    }
    rec.push_back(r0);
    rec.push_back(r1);
    return true;
}

// Elements of odd total multiplicity in a and b: the sum over GF(2) of two
// sets of symbols or records.
static std::vector<uint32_t> xor_sets(std::vector<uint32_t> a, const std::vector<uint32_t> &b) {
    a.insert(a.end(), b.begin(), b.end());
    std::sort(a.begin(), a.end());
    std::vector<uint32_t> r;
    for (size_t i = 0; i < a.size();) {
        size_t j = i;
        while (j < a.size() && a[j] == a[i]) ++j;
        if ((j - i) & 1) r.push_back(a[i]);
        i = j;
    }
    return r;
}

// Caps on a folded node's expression (they bound the pushes and flip entries
// that folding adds).
static const size_t FOLD_MAX_PREDS = 64, FOLD_MAX_NOISE = 1024;

namespace {
struct Node {
    uint8_t cst = 0, rm = 0, sec = 0;
    uint32_t row = FR_NO_ROW, rm_t = 0;  // rm_t: the measurement whose RandomMeas word is added
    std::vector<uint32_t> preds, succs, noise;
    int emit = -1, first = 1 << 30, slot = -1;
};
struct Step {
    uint32_t kind;
    uint32_t cls, r0, r1;
    std::vector<uint32_t> nodes;
};
}  // namespace

// The wave-owned schedule from the step schedule.  The steps keep their order
// (so every slot interval of the colouring holds); consecutive EMIT steps'
// nodes are packed into batches of up to 64 as long as no node depends on a
// node already in the batch (a node reads its slot before any push of its
// batch lands, so a dependency inside a batch would be lost).  A NOISE step
// ends the batch before it.  Batches are staged in order; a batch that does
// not fit the rest of the staging buffer first flushes it.
static void build_wave_ops(const std::vector<Step> &steps, const std::vector<uint32_t> &first_node,
                           const std::vector<Node> &nd, FrameSchedule &F) {
    F.wops.clear();
    F.wrows.clear();
    std::vector<int64_t> in_batch(nd.size(), -1);
    int64_t batch_id = 0;
    uint32_t b_first = 0, b_n = 0, pos = 0, buf = 0, flush_off = 0;
    std::vector<uint32_t> staged;  // rows staged in the open buffer
    auto op = [&](std::initializer_list<uint32_t> w) {
        std::vector<uint32_t> r(w);
        r.resize(WV_OP_WORDS, 0);
        F.wops.insert(F.wops.end(), r.begin(), r.end());
    };
    auto flush = [&]() {
        if (staged.empty()) return;
        op({WV_FLUSH, flush_off, (uint32_t)staged.size(), buf});
        F.wrows.insert(F.wrows.end(), staged.begin(), staged.end());
        flush_off += (uint32_t)staged.size();
        staged.clear();
        pos = 0;
        buf ^= 1u;
        F.w_n_flushes += 1;
    };
    auto close = [&]() {
        if (!b_n) return;
        if (pos + b_n > WV_STAGE_ROWS) flush();
        op({WV_BATCH, b_first, b_n, pos, buf, 0, 0});
        for (uint32_t i = 0; i < b_n; ++i) staged.push_back(0);  // rows filled below
        pos += b_n;
        b_n = 0;
        ++batch_id;
        F.w_n_batches += 1;
    };
    std::vector<uint32_t> rec_of_node(nd.size(), 0);  // node id -> record index
    for (size_t i = 0; i < steps.size(); ++i) {
        const Step &st = steps[i];
        if (st.kind == FR_NOISE) {
            close();
            op({WV_NOISE, st.cls, st.r1, 0, 0});  // step index and next class filled below
            continue;
        }
        for (size_t k = 0; k < st.nodes.size(); ++k) {
            const uint32_t id = st.nodes[k];
            const uint32_t rec = first_node[i] + (uint32_t)k;
            rec_of_node[id] = rec;
            bool dep = false;
            for (uint32_t u : nd[id].preds) dep |= in_batch[u] == batch_id;
            if (b_n && (b_n == WV_BATCH_MAX || dep || rec != b_first + b_n)) close();
            if (!b_n) b_first = rec;
            in_batch[id] = batch_id;
            ++b_n;
        }
    }
    close();
    flush();
    // staged rows, the NOISE steps' local indices and look-ahead fields
    std::vector<uint32_t> row_of_rec(F.nodes.size() / 8);
    for (size_t r = 0; r < row_of_rec.size(); ++r) row_of_rec[r] = F.nodes[8 * r + 1];
    {
        size_t fo = 0;
        std::vector<uint32_t> batch_rows;
        for (size_t o = 0; o < F.wops.size(); o += WV_OP_WORDS) {
            const uint32_t *w = &F.wops[o];
            if (w[0] == WV_BATCH)
                for (uint32_t q = 0; q < w[2]; ++q) batch_rows.push_back(row_of_rec[w[1] + q]);
            if (w[0] == WV_FLUSH) {
                for (uint32_t q = 0; q < w[2]; ++q) F.wrows[fo + q] = batch_rows[q];
                batch_rows.erase(batch_rows.begin(), batch_rows.begin() + w[2]);
                fo += w[2];
            }
        }
    }
    std::map<uint32_t, uint32_t> next_local;
    for (size_t o = 0; o < F.wops.size(); o += WV_OP_WORDS)
        if (F.wops[o] == WV_NOISE) F.wops[o + 3] = next_local[F.wops[o + 1]]++;
    uint32_t nn_cls = FR_NONE, nb_first = 0, nb_n = 0;
    for (size_t o = F.wops.size(); o >= WV_OP_WORDS;) {
        o -= WV_OP_WORDS;
        uint32_t *w = &F.wops[o];
        if (w[0] == WV_NOISE) {
            w[4] = nn_cls;
            nn_cls = w[1];
        } else if (w[0] == WV_BATCH) {
            w[5] = nb_first;
            w[6] = nb_n;
            nb_first = w[1];
            nb_n = w[2];
        }
    }
    F.w_first_noise_cls = nn_cls;
    F.w_first_batch[0] = nb_first;
    F.w_first_batch[1] = nb_n;
    F.wave_ok = true;
}

void build_frame_schedule(const Program &P, FrameSchedule &F) {
    F = FrameSchedule();
    if (P.k_max != 0) return;
    uint64_t fl_total = 0;
    for (const Channel &ch : P.chans) fl_total += ch.J;
    if (fl_total >= (1u << 26)) return;  // event records hold 26-bit flip-table indices
    for (const NoiseClass &nc : P.classes)
        if (nc.chans.size() > (1u << 25)) return;  // class stream positions are 32-bit
    uint64_t thr_total = 0;
    for (const Channel &ch : P.chans) thr_total += ch.thr.size();
    if (thr_total >= (1u << 23)) return;  // channel records hold 23-bit threshold offsets
    const uint32_t M = (uint32_t)P.n_meas, D = (uint32_t)P.n_det, B = (uint32_t)P.n_obs;
    const uint32_t NN = M + D + B;
    std::vector<Node> nd(NN);
    for (uint32_t t = 0; t < M; ++t) {
        const Instr &I = P.instrs[(size_t)P.meas_instr[t]];
        Node &v = nd[t];
        if (I.kind == RANDOM_MEAS) {
            v.rm = 1;
            v.rm_t = t;
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
    std::vector<Step> steps;
    std::vector<int> chan_step(P.chans.size(), -1);
    std::map<uint32_t, std::pair<uint32_t, uint32_t>> seg;  // class -> rank range
    std::vector<uint32_t> seg_chans;
    std::vector<uint32_t> level;
    std::vector<uint8_t> in_level(NN, 0);
    // v's expression with every dependency on the open level replaced by that
    // node's expression; false (v unchanged) past the caps or where two
    // different RandomMeas words would meet.  A node of the level depends on no
    // other node of it, and the nodes it depends on precede it, so each
    // replacement removes one dependency on the level.
    auto fold = [&](Node &v) -> bool {
        std::vector<uint32_t> preds = xor_sets(v.preds, {}), noise = xor_sets(v.noise, {});
        uint8_t cst = v.cst, rm = v.rm;
        uint32_t rm_t = v.rm_t;
        for (;;) {
            int64_t u = -1;
            for (uint32_t x : preds)
                if (in_level[x]) u = x;
            if (u < 0) break;
            const Node &a = nd[(size_t)u];
            if (a.rm) {
                if (rm && rm_t != a.rm_t) return false;
                rm_t = a.rm_t;
                rm ^= 1;
            }
            cst ^= a.cst;
            preds = xor_sets(xor_sets(preds, {(uint32_t)u}), a.preds);
            noise = xor_sets(noise, a.noise);
            if (preds.size() > FOLD_MAX_PREDS || noise.size() > FOLD_MAX_NOISE) return false;
        }
        v.preds = preds;
        v.noise = noise;
        v.cst = cst;
        v.rm = rm;
        v.rm_t = rm ? rm_t : 0;
        return true;
    };
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
    // a level of independent nodes is emitted in chunks of at most FR_LEVEL_MAX
    auto flush_level = [&]() {
        if (level.empty()) return;
        for (size_t i0 = 0; i0 < level.size(); i0 += FR_LEVEL_MAX) {
            Step s;
            s.kind = FR_EMIT;
            s.cls = s.r0 = s.r1 = 0;
            s.nodes.assign(level.begin() + i0, level.begin() + std::min(level.size(), i0 + FR_LEVEL_MAX));
            steps.push_back(s);
            for (uint32_t v : s.nodes) {
                nd[v].emit = (int)steps.size() - 1;
                in_level[v] = 0;
            }
        }
        F.max_level = std::max<uint32_t>(F.max_level, (uint32_t)level.size());
        level.clear();
    };
    // Channels wait (pending) until a node that reads one of them arrives: a
    // class's stream is consumed in rank order, so the pending channels of a
    // class are a contiguous rank range, and nodes that read none of them
    // (detectors, records of other qubits) join the open level.  When a node
    // reads a pending channel, the open level is emitted and the NOISE steps
    // follow -- unless no node of the level takes any contribution (random
    // outcomes with nothing added): such a level holds no slots, so it stays
    // open behind the NOISE steps, which its nodes do not read.
    std::vector<int32_t> sym_chan_of(P.n_noise_sym, -1);
    for (uint32_t c = 0; c < P.chans.size(); ++c)
        for (uint32_t k = 0; k < P.chans[c].nsym; ++k) sym_chan_of[P.chans[c].sym0 + k] = (int32_t)c;
    std::vector<uint8_t> pending(P.chans.size(), 0);
    auto flush_pending = [&]() {
        for (uint32_t c : seg_chans) pending[c] = 0;
        flush_noise();
    };
    for (const Item &it : items) {
        if (it.kind == 0) {
            const Channel &ch = P.chans[it.id];
            auto f = seg.find((uint32_t)ch.cls);
            if (f == seg.end()) seg[(uint32_t)ch.cls] = {(uint32_t)ch.rank, (uint32_t)ch.rank + 1};
            else f->second.second = (uint32_t)ch.rank + 1;
            seg_chans.push_back(it.id);
            pending[it.id] = 1;
        } else {
            bool reads = false;
            for (uint32_t sy : nd[it.id].noise) {
                const int32_t c = sym_chan_of[sy];
                reads |= c >= 0 && pending[(size_t)c];
            }
            if (reads) {
                bool holds = false;
                for (uint32_t u : level) holds |= !nd[u].preds.empty() || !nd[u].noise.empty();
                if (holds) flush_level();
                flush_pending();
            }
            bool dep = false;
            for (uint32_t u : nd[it.id].preds) dep |= in_level[u] != 0;
            if (dep && !fold(nd[it.id])) flush_level();
            level.push_back(it.id);
            in_level[it.id] = 1;
        }
    }
    flush_level();
    flush_pending();
    for (uint32_t i = 0; i < NN; ++i)
        for (uint32_t u : nd[i].preds) nd[u].succs.push_back(i);

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
    if (n_slots >= (1u << 16)) return;  // flip entries hold 16-bit slots
    F.rec_ok = n_slots < (1u << 12);  // the step kernel's entries hold 12-bit slots
    // noise symbol -> consumer slots; (channel, branch) -> slots flipped
    std::vector<std::vector<uint32_t>> cons(P.n_noise_sym);
    for (uint32_t i = 0; i < NN; ++i)
        for (uint32_t s : nd[i].noise) cons[s].push_back((uint32_t)nd[i].slot);
    std::vector<uint64_t> chan_fl(P.chans.size(), 0), chan_thr(P.chans.size(), 0);
    std::vector<double> chan_k1(P.chans.size(), 0), chan_k2(P.chans.size(), 0);  // E[entries], E[entries^2] per event
    std::vector<double> chan_f1(P.chans.size(), 0), chan_f2(P.chans.size(), 0);  // E[slot flips], E[flips^2] per event
    uint64_t thr_off = 0;
    for (size_t c = 0; c < P.chans.size(); ++c) {
        const Channel &ch = P.chans[c];
        chan_thr[c] = thr_off;
        thr_off += ch.thr.size();
        chan_fl[c] = F.frec.size() / 2;
        for (uint32_t j = 0; j < ch.J; ++j) {
            std::map<uint32_t, int> par;
            for (uint32_t i = 0; i < ch.nsym; ++i)
                if ((ch.bmask[j] >> i) & 1u)
                    for (uint32_t sl : cons[ch.sym0 + i]) par[sl] ^= 1;
            std::vector<uint32_t> fl;
            for (auto &kv : par)
                if (kv.second) fl.push_back(kv.first);
            F.n_flips += fl.size();
            if (!pack_record(fl, F.frec, F.fl3)) return;
            if (fl.size() <= 3 && !fl.empty()) {
                uint64_t w = fl.size();
                for (size_t q = 0; q < fl.size(); ++q) w |= (uint64_t)fl[q] << (16 + 16 * q);
                F.wfl.push_back(w);
            } else {
                F.wfl.push_back(((uint64_t)fl.size() << 8) | ((uint64_t)F.wsl.size() << 32));
                for (uint32_t sl : fl) F.wsl.push_back((uint16_t)sl);
            }
            // branch probability under the draw contract
            double pj = 1.0 / ch.J;
            if (!ch.uniform) {
                const double lo = j ? (double)ch.thr[j - 1] : 0.0;
                pj = ((double)ch.thr[j] - lo) / 4294967296.0;
            }
            const double k = (double)((fl.size() + 3) / 4);
            chan_k1[c] += pj * k;
            chan_k2[c] += pj * k * k;
            const double f = (double)fl.size();
            chan_f1[c] += pj * f;
            chan_f2[c] += pj * f * f;
        }
    }
    // step index of every channel within its class
    std::vector<uint32_t> chan_step_local(P.chans.size(), 0);
    {
        std::vector<uint32_t> next_local(P.classes.size(), 0);
        for (const Step &st : steps) {
            if (st.kind != FR_NOISE) continue;
            const uint32_t sl = next_local[st.cls]++;
            if (sl > 255) return;  // flip entries hold 8-bit step indices
            for (uint32_t r = st.r0; r < st.r1; ++r) chan_step_local[(size_t)P.classes[st.cls].chans[r]] = sl;
        }
    }
    F.ltab_ok = true;
    // channel record per (class, rank): flip-table offset | J << 26 | uniform << 32 |
    // step index << 33 | threshold offset << 41; per-class flip-entry capacity per
    // word: the expected count plus 8 standard deviations (compound Poisson) plus 64
    for (const NoiseClass &nc : P.classes) {
        double m1 = 0, m2 = 0, f1 = 0, f2 = 0;
        const double p = std::ldexp((double)nc.p32, -32);
        for (int32_t c : nc.chans) {
            const Channel &ch = P.chans[(size_t)c];
            F.chinfo.push_back(chan_fl[(size_t)c] | ((uint64_t)ch.J << 26) | ((uint64_t)ch.uniform << 32) |
                               ((uint64_t)chan_step_local[(size_t)c] << 33) | (chan_thr[(size_t)c] << 41));
            // compact record for the LDS copy of the walk tables: flip-table offset | J << 20
            F.ltab_ok = F.ltab_ok && ch.uniform && chan_fl[(size_t)c] < (1u << 20) && ch.J < 64;
            F.ci32.push_back((uint32_t)(chan_fl[(size_t)c] & 0xFFFFFu) | ((uint32_t)ch.J << 20));
            F.st8.push_back((uint8_t)chan_step_local[(size_t)c]);
            m1 += 64.0 * p * chan_k1[(size_t)c];
            m2 += 64.0 * p * chan_k2[(size_t)c];
            f1 += 64.0 * p * chan_f1[(size_t)c];
            f2 += 64.0 * p * chan_f2[(size_t)c];
        }
        F.events_per_word += (double)nc.chans.size() * 64.0 * p;
        const double cap = std::ceil((m1 + 8.0 * std::sqrt(m2) + 64.0) / 64.0) * 64.0;
        F.cls_cap.push_back((uint32_t)std::min(cap, 16777216.0));
        const double wcap = std::ceil((f1 + 8.0 * std::sqrt(f2) + 64.0) / 64.0) * 64.0;
        F.wcap.push_back((uint32_t)std::min(wcap, 16777216.0));
    }
    // the LDS copy moves whole 16-byte units: both compact arrays padded to a multiple of 16 channels
    F.ci32.resize((F.ci32.size() + 15) & ~(size_t)15, 0u);
    F.st8.resize(F.ci32.size(), 0u);
    // encode steps (FR_STEP_WORDS per step, see launch_args.hpp) and node records
    std::vector<uint32_t> first_node(steps.size(), 0);
    uint32_t nodes_so_far = 0;
    for (size_t i = 0; i < steps.size(); ++i) {
        first_node[i] = nodes_so_far;
        if (steps[i].kind == FR_EMIT) nodes_so_far += (uint32_t)steps[i].nodes.size();
    }
    uint32_t ne_first = 0, ne_n = 0, nn_cls = FR_NONE;  // next EMIT / NOISE step after the current one
    std::vector<uint32_t> rec(steps.size() * FR_STEP_WORDS, 0);
    for (size_t i = steps.size(); i-- > 0;) {
        const Step &s = steps[i];
        uint32_t *r = &rec[i * FR_STEP_WORDS];
        r[0] = s.kind;
        if (s.kind == FR_NOISE) {
            r[1] = s.cls;
            r[2] = s.r1;
            r[3] = s.r0 < s.r1 ? chan_step_local[(size_t)P.classes[s.cls].chans[s.r0]] : 0u;
        } else {
            r[1] = first_node[i];
            r[2] = (uint32_t)s.nodes.size();
        }
        r[5] = ne_first;
        r[6] = ne_n;
        r[7] = nn_cls;
        if (s.kind == FR_EMIT) {
            ne_first = first_node[i];
            ne_n = (uint32_t)s.nodes.size();
        } else {
            nn_cls = s.cls;
        }
    }
    F.steps = rec;
    F.first_emit = {ne_first, ne_n};
    F.first_noise_cls = nn_cls;
    for (const Step &s : steps) {
        if (s.kind != FR_EMIT) continue;
        for (uint32_t id : s.nodes) {
            const Node &v = nd[id];
            uint32_t flags = (v.cst ? 1u : 0u) | (v.slot >= 0 ? 2u : 0u) | (v.rm ? 4u : 0u) | ((uint32_t)v.sec << 4);
            const uint32_t np = (uint32_t)v.succs.size();
            F.nodes.push_back((v.slot >= 0 ? (uint32_t)v.slot : F.n_slots) | (flags << 24));
            F.nodes.push_back(v.row);
            F.nodes.push_back(v.rm_t);
            F.nodes.push_back(np);
            F.nodes.push_back(np > 0 ? (uint32_t)nd[v.succs[0]].slot : 0u);
            F.nodes.push_back(np > 1 ? (uint32_t)nd[v.succs[1]].slot : 0u);
            F.nodes.push_back((uint32_t)F.push.size());  // pushes beyond the first two
            F.nodes.push_back(v.rm ? (uint32_t)F.rm_meas.size() : 0u);  // RandomMeas index (wave kernel)
            if (v.rm) F.rm_meas.push_back(v.rm_t);
            for (uint32_t k = 2; k < np; ++k) F.push.push_back((uint32_t)nd[v.succs[k]].slot);
            // compact record (step-synchronous kernel), 4 words: slot | flags << 12 | push count << 20, row,
            // two successor slots (12 bits each), offset into push16 (a RandomMeas node's measurement first,
            // then its successors past the first two)
            const uint32_t sl = v.slot >= 0 ? (uint32_t)v.slot : F.n_slots;
            if (sl >= (1u << 12) || np >= (1u << 12)) F.rec_ok = false;
            F.nodes16.push_back(sl | (flags << 12) | (np << 20));
            F.nodes16.push_back(v.row);
            F.nodes16.push_back((np > 0 ? (uint32_t)nd[v.succs[0]].slot : 0u) |
                                ((np > 1 ? (uint32_t)nd[v.succs[1]].slot : 0u) << 12));
            F.nodes16.push_back((uint32_t)F.push16.size());
            if (v.rm) F.push16.push_back(v.rm_t);
            for (uint32_t k = 2; k < np; ++k) F.push16.push_back((uint32_t)nd[v.succs[k]].slot);
        }
    }
    F.n_pushes = 0;
    for (uint32_t i = 0; i < NN; ++i) F.n_pushes += nd[i].succs.size();
    F.n_steps = steps.size();
    F.ok = F.n_steps > 0;
    build_wave_ops(steps, first_node, nd, F);
}

}  // namespace symft
