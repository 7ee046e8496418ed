// State-flow graph construction and the four inter-kernel passes of the
// paper's Section 6: activation demotion (6.3), list generation removal
// (6.2), dead store elimination (6.5) and task fusion (6.4 with the criteria
// of supplement Section 2).
#include "sfg.hpp"

#include <algorithm>
#include <cstring>
#include <queue>

namespace ats {

namespace {

inline uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h * 0xff51afd7ed558ccdull;
}

inline StateKey VAL(uint64_t g, int ch) { return {g, ch, ST_VALUE}; }
inline StateKey MASK(uint64_t g) { return {g, -1, ST_MASK}; }
inline StateKey LIST(uint64_t g) { return {g, -1, ST_LIST}; }
inline StateKey ALLOC(uint64_t g) { return {g, -1, ST_ALLOC}; }
inline StateKey EXT(const void *p) { return {(uint64_t)(uintptr_t)p, -1, ST_EXT}; }

bool is_particle_kind(int k) {
    return k == AT_TASK_ADVECT || k == AT_TASK_P2G || k == AT_TASK_G2P || k == AT_TASK_P2G_MLS ||
           k == AT_TASK_G2P_APIC;
}
bool is_mpm_kind(int k) { return k == AT_TASK_P2G_MLS || k == AT_TASK_G2P_APIC; }
bool is_scatter_kind(int k) { return k == AT_TASK_P2G || k == AT_TASK_P2G_MLS; }

bool is_tiled_stencil(int op) {
    return op == AT_OP_LAP_UPDATE || op == AT_OP_JACOBI || op == AT_OP_DIFFUSE || op == AT_OP_DIFFUSE_ADJ;
}

int op_nch(int op) {
    switch (op) {
    case AT_OP_LAP_UPDATE: return 2;
    case AT_OP_AXPY: return 2;
    case AT_OP_JACOBI: return 3;
    case AT_OP_COPY: return 2;
    case AT_OP_FILL: return 1;   // at least one
    case AT_OP_INC: return 1;
    case AT_OP_DIFFUSE: return 3;
    case AT_OP_DIFFUSE_ADJ: return 5;
    case AT_OP_NORMALISE: return 3;
    case AT_OP_ADVECT: return 3;
    case AT_OP_MACCORMACK: return 5;
    case AT_OP_MPM_GRID: return 3;
    default: return -1;
    }
}

// Accesses of one member task (Section 4, "Tasks": input and output states).
void member_accesses(const at_task &t, const Member &mb, bool check, int16_t mi, std::vector<Access> &acc) {
    const at_grid_s *g = task_grid(t);
    const uint64_t gu = g ? g->uid : 0;
    const bool ptr_root = g && g->desc.root_kind == AT_ROOT_POINTER;
    auto add = [&](StateKey s, uint8_t mode, uint8_t pat, uint8_t fl) { acc.push_back({s, mode, pat, fl, mi}); };
    const uint8_t U = F_UNIQUE;
    switch (t.kind) {
    case AT_TASK_ACTIVATE:
        add(EXT(t.ext[0]), M_R, P_ELEM, 0);
        add(MASK(gu), M_R | M_W, P_SCATTER, F_ACTIVATING);
        if (ptr_root) add(ALLOC(gu), M_R | M_W, P_SCATTER, F_ACTIVATING);
        break;
    case AT_TASK_LISTGEN:
        add(MASK(gu), M_R, P_ELEM, 0);
        add(LIST(gu), M_W, P_ELEM, F_FULL);
        break;
    case AT_TASK_STENCIL: {
        add(LIST(gu), M_R, P_ELEM, 0);
        const int32_t *c = t.ch;
        bool stencil_read = false, writes = false;
        auto rd = [&](int ch, bool st) {
            add(VAL(gu, ch), M_R, st ? P_STENCIL : P_ELEM, st ? 0 : U);
            stencil_read |= st;
        };
        auto wr = [&](int ch, bool full, bool also_read) {
            add(VAL(gu, ch), also_read ? (M_R | M_W) : M_W, P_ELEM, U | (full ? F_FULL : 0));
            writes = true;
        };
        switch (t.op) {
        case AT_OP_LAP_UPDATE: rd(c[0], true); wr(c[1], true, false); break;
        case AT_OP_AXPY: rd(c[1], false); wr(c[0], false, true); break;
        case AT_OP_JACOBI: rd(c[0], true); rd(c[1], false); wr(c[2], true, false); break;
        case AT_OP_COPY: rd(c[1], false); wr(c[0], true, false); break;
        case AT_OP_FILL:
            for (int q = 0; q < 7; ++q)
                if (c[q] >= 0 && ((mb.keep >> q) & 1u)) wr(c[q], true, false);
            break;
        case AT_OP_INC: wr(c[0], false, true); break;
        case AT_OP_DIFFUSE: rd(c[0], true); rd(c[1], true); wr(c[2], true, false); break;
        case AT_OP_DIFFUSE_ADJ:
            rd(c[0], true); rd(c[1], true); rd(c[2], true);
            wr(c[3], true, false); wr(c[4], false, true);
            break;
        case AT_OP_ADVECT:
            // q at back-traced points (any offset); v at the voxel, and along
            // the path with the RK3 back-trace
            rd(c[0], true);
            for (int q = 0; q < 3; ++q) rd(c[1] + q, t.param[1] != 0.f);
            wr(c[2], true, false);
            break;
        case AT_OP_MACCORMACK:
            // q at the corners of the back-traced point and at the voxel
            rd(c[0], true);
            for (int q = 0; q < 3; ++q) rd(c[1] + q, t.param[1] != 0.f);
            rd(c[2], false);
            rd(c[3], false);
            wr(c[4], true, false);
            break;
        case AT_OP_NORMALISE:
            rd(c[0], false);
            for (int q = 0; q < 3; ++q) rd(c[1] + q, false);
            for (int q = 0; q < 3; ++q)
                if ((mb.keep >> q) & 1u) wr(c[2] + q, true, false);
            break;
        case AT_OP_MPM_GRID:
            rd(c[0], false);
            for (int q = 0; q < 3; ++q) rd(c[1] + q, false);
            for (int q = 0; q < 3; ++q) wr(c[2] + q, true, false);
            break;
        default: break;
        }
        if (stencil_read) add(MASK(gu), M_R, P_STENCIL, 0);
        if (check && writes) {
            // activation on write at the loop index: a (usually false)
            // modification of the mask state (Section 6.3)
            add(MASK(gu), M_R | M_W, P_ELEM, F_ACTIVATING | U);
            if (ptr_root) add(ALLOC(gu), M_R | M_W, P_ELEM, F_ACTIVATING | U);
        }
        break;
    }
    case AT_TASK_ADVECT: {
        const uint8_t u = (t.flags & AT_TASKF_LOOP_UNIQUE) ? U : 0;
        add(EXT(t.ext[1]), M_R, P_ELEM, u);
        add(EXT(t.ext[0]), M_R | M_W, P_ELEM, u);
        break;
    }
    case AT_TASK_P2G: {
        const uint8_t u = (t.flags & AT_TASKF_LOOP_UNIQUE) ? U : 0;
        add(EXT(t.ext[0]), M_R, P_ELEM, u);
        add(EXT(t.ext[1]), M_R, P_ELEM, u);
        add(EXT(t.ext[2]), M_R, P_ELEM, u);
        add(VAL(gu, t.ch[0]), M_R | M_W, P_SCATTER, 0);
        for (int q = 0; q < 3; ++q) add(VAL(gu, t.ch[1] + q), M_R | M_W, P_SCATTER, 0);
        if (t.op == AT_ACT_NONE) {
            add(MASK(gu), M_R, P_GATHER, 0);   // reads the roots, activates nothing
        } else {
            add(MASK(gu), M_R | M_W, P_SCATTER, F_ACTIVATING);
            if (ptr_root) add(ALLOC(gu), M_R | M_W, P_SCATTER, F_ACTIVATING);
        }
        break;
    }
    case AT_TASK_G2P: {
        const uint8_t u = (t.flags & AT_TASKF_LOOP_UNIQUE) ? U : 0;
        add(EXT(t.ext[0]), M_R, P_ELEM, u);
        for (int q = 0; q < 3; ++q) add(VAL(gu, t.ch[0] + q), M_R, P_GATHER, 0);
        add(MASK(gu), M_R, P_GATHER, 0);
        add(EXT(t.ext[1]), M_W, P_ELEM, u | F_FULL);
        break;
    }
    case AT_TASK_P2G_MLS: {
        const uint8_t u = (t.flags & AT_TASKF_LOOP_UNIQUE) ? U : 0;
        add(EXT(t.ext[0]), M_R, P_ELEM, u);
        add(EXT(t.ext[1]), M_R, P_ELEM, u);
        add(EXT(t.ext[2]), M_R, P_ELEM, u);
        add(EXT(t.ext[3]), M_R | M_W, P_ELEM, u);
        add(VAL(gu, t.ch[0]), M_R | M_W, P_SCATTER, 0);
        for (int q = 0; q < 3; ++q) add(VAL(gu, t.ch[1] + q), M_R | M_W, P_SCATTER, 0);
        if (t.op == AT_ACT_NONE) {
            add(MASK(gu), M_R, P_GATHER, 0);
        } else {
            add(MASK(gu), M_R | M_W, P_SCATTER, F_ACTIVATING);
            if (ptr_root) add(ALLOC(gu), M_R | M_W, P_SCATTER, F_ACTIVATING);
        }
        break;
    }
    case AT_TASK_G2P_APIC: {
        // keep bit 0: the store of v; bit 1: the store of C (dead store
        // elimination clears them; the gather itself always runs)
        const uint8_t u = (t.flags & AT_TASKF_LOOP_UNIQUE) ? U : 0;
        add(EXT(t.ext[0]), M_R, P_ELEM, u);
        for (int q = 0; q < 3; ++q) add(VAL(gu, t.ch[0] + q), M_R, P_GATHER, 0);
        add(MASK(gu), M_R, P_GATHER, 0);
        if (mb.keep & 1u) add(EXT(t.ext[1]), M_W, P_ELEM, u | F_FULL);
        if (mb.keep & 2u) add(EXT(t.ext[2]), M_W, P_ELEM, u | F_FULL);
        break;
    }
    case AT_TASK_RESTRICT: {
        // fine values at the loop index; coarse values at I/2 (8 iterations
        // per coarse voxel); the coarse mask is written when activating
        const at_grid_s *c = reinterpret_cast<const at_grid_s *>(t.grid2);
        add(LIST(gu), M_R, P_ELEM, 0);
        add(VAL(gu, t.ch[0]), M_R, P_ELEM, U);
        add(VAL(c->uid, t.ch[1]), M_R | M_W, P_SCATTER, 0);
        if (check) {
            add(MASK(c->uid), M_R | M_W, P_SCATTER, F_ACTIVATING);
            if (c->desc.root_kind == AT_ROOT_POINTER) add(ALLOC(c->uid), M_R | M_W, P_SCATTER, F_ACTIVATING);
        } else {
            add(MASK(c->uid), M_R, P_GATHER, 0);
        }
        break;
    }
    case AT_TASK_PROLONG: {
        const at_grid_s *c = reinterpret_cast<const at_grid_s *>(t.grid2);
        add(LIST(gu), M_R, P_ELEM, 0);
        add(VAL(c->uid, t.ch[0]), M_R, P_GATHER, 0);
        add(MASK(c->uid), M_R, P_GATHER, 0);
        add(VAL(gu, t.ch[1]), M_R | M_W, P_ELEM, U);
        if (check) {
            add(MASK(gu), M_R | M_W, P_ELEM, F_ACTIVATING | U);
            if (ptr_root) add(ALLOC(gu), M_R | M_W, P_ELEM, F_ACTIVATING | U);
        }
        break;
    }
    default: break;
    }
}

// The graph rebuilt from a topological order (Section 4.2).
struct Sim {
    int n = 0, words = 0;
    std::vector<uint64_t> adj;        // adj[i*words + j/64] bit j%64: edge i -> j
    std::vector<uint64_t> list_ver;   // struct-for: version of the list it loops over
    std::vector<uint64_t> mask_at;    // listgen: version of the mask it reads
    std::vector<uint64_t> act_sig;    // activate: identity of the activation
    std::unordered_map<StateKey, uint64_t, StateKeyHash> cur;
    bool edge(int i, int j) const { return (adj[(size_t)i * words + (j >> 6)] >> (j & 63)) & 1ull; }
    void set(int i, int j) { adj[(size_t)i * words + (j >> 6)] |= 1ull << (j & 63); }
};

// Identity of a restriction's activation: the coarse parents of the blocks
// of one version of the fine grid's list.
uint64_t restrict_sig(const at_task &t, uint64_t list_ver) {
    uint64_t h = mix(0x52ull, reinterpret_cast<const at_grid_s *>(t.grid)->uid);
    h = mix(h, reinterpret_cast<const at_grid_s *>(t.grid2)->uid);
    return mix(h, list_ver);
}

uint64_t activation_sig(const at_task &t, uint64_t ext_ver) {
    const at_grid_s *g = task_grid(t);
    uint64_t h = mix(0x51ull, g ? g->uid : 0);
    h = mix(h, (uint64_t)(uint32_t)t.op);
    h = mix(h, (uint64_t)(uintptr_t)t.ext[0]);
    h = mix(h, ext_ver);
    return mix(h, (uint64_t)t.n);
}

Sim simulate(const std::vector<Node> &nodes, const at_task *tasks, const Persist &P) {
    Sim S;
    S.n = (int)nodes.size();
    S.words = (S.n + 63) / 64;
    S.adj.assign((size_t)S.n * S.words, 0);
    S.list_ver.assign(S.n, 0);
    S.mask_at.assign(S.n, 0);
    S.act_sig.assign(S.n, 0);
    // dense index of the window's states: one hash lookup per access
    std::unordered_map<StateKey, int, StateKeyHash> id;
    id.reserve(nodes.size() * 8);
    std::vector<StateKey> keys;
    std::vector<uint64_t> cur;
    std::vector<char> touched;   // versions the simulation reads or bumps (reported in S.cur)
    std::vector<int> last_writer;
    std::vector<std::vector<int>> readers;
    auto sidx = [&](const StateKey &s) -> int {
        auto it = id.find(s);
        if (it != id.end()) return it->second;
        const int k = (int)keys.size();
        id.emplace(s, k);
        keys.push_back(s);
        cur.push_back(P.ver(s));
        touched.push_back(0);
        last_writer.push_back(-1);
        readers.emplace_back();
        return k;
    };
    std::vector<int> written;
    for (int i = 0; i < S.n; ++i) {
        const Node &nd = nodes[i];
        const at_task &t0 = tasks[nd.members[0].task];
        auto version_of = [&](const StateKey &s) -> uint64_t {
            const int k = sidx(s);
            touched[k] = 1;
            return cur[k];
        };
        if (nd.loop == LT_STRUCT) S.list_ver[i] = version_of(LIST(nd.loop_grid));
        if (t0.kind == AT_TASK_LISTGEN) S.mask_at[i] = version_of(MASK(task_grid(t0)->uid));
        if (t0.kind == AT_TASK_ACTIVATE) S.act_sig[i] = activation_sig(t0, version_of(EXT(t0.ext[0])));
        if (t0.kind == AT_TASK_RESTRICT) S.act_sig[i] = restrict_sig(t0, S.list_ver[i]);
        for (const Access &a : nd.acc) {
            if (!(a.mode & M_R)) continue;
            const int k = sidx(a.s);
            if (last_writer[k] >= 0 && last_writer[k] != i) S.set(last_writer[k], i);
            auto &rv = readers[k];
            if (rv.empty() || rv.back() != i) rv.push_back(i);
        }
        written.clear();
        for (const Access &a : nd.acc) {
            if (!(a.mode & M_W)) continue;
            const int k = sidx(a.s);
            if (std::find(written.begin(), written.end(), k) != written.end()) continue;
            written.push_back(k);
            if (last_writer[k] >= 0 && last_writer[k] != i) S.set(last_writer[k], i);
            auto &rv = readers[k];
            for (int r : rv)
                if (r != i) S.set(r, i);
            rv.clear();
            last_writer[k] = i;
            cur[k] += 1;
            touched[k] = 1;
        }
    }
    S.cur.reserve(keys.size());
    for (size_t k = 0; k < keys.size(); ++k)
        if (touched[k]) S.cur.emplace(keys[k], cur[k]);
    return S;
}

// reach[i] = nodes reachable from i by a path of length >= 1.
std::vector<uint64_t> closure(const Sim &S) {
    std::vector<uint64_t> reach(S.adj);
    for (int i = S.n - 1; i >= 0; --i) {
        uint64_t *ri = &reach[(size_t)i * S.words];
        for (int w = 0; w < S.words; ++w) {
            uint64_t bits = S.adj[(size_t)i * S.words + w];
            while (bits) {
                const int j = w * 64 + __builtin_ctzll(bits);
                bits &= bits - 1;
                const uint64_t *rj = &reach[(size_t)j * S.words];
                for (int q = 0; q < S.words; ++q) ri[q] |= rj[q];
            }
        }
    }
    return reach;
}

inline bool bit(const std::vector<uint64_t> &m, int words, int i, int j) {
    return (m[(size_t)i * words + (j >> 6)] >> (j & 63)) & 1ull;
}

bool node_has_kind(const Node &nd, const at_task *tasks, int kind) {
    for (const Member &m : nd.members)
        if (tasks[m.task].kind == kind) return true;
    return false;
}

}  // namespace

size_t StateKeyHash::operator()(const StateKey &k) const {
    return (size_t)mix(mix(k.obj, (uint64_t)(uint32_t)k.ch), k.kind);
}

void Persist::forget_grid(uint64_t uid) {
    for (auto it = version.begin(); it != version.end();) {
        if (it->first.kind != ST_EXT && it->first.obj == uid) it = version.erase(it);
        else ++it;
    }
    list_src.erase(uid);
    act_sigs.erase(uid);
}

void Persist::deactivate_grid(uint64_t uid) {
    for (auto &kv : version)
        if (kv.first.kind != ST_EXT && kv.first.obj == uid) kv.second += 1;
    version[MASK(uid)] += 0;   // make sure the mask has an entry
    version[MASK(uid)] += 1;
    version[LIST(uid)] += 1;
    list_src.erase(uid);
    act_sigs.erase(uid);
}

const at_grid_s *task_grid(const at_task &t) { return reinterpret_cast<const at_grid_s *>(t.grid); }

std::string validate_task(const at_task &t) {
    const bool two_level = t.kind == AT_TASK_RESTRICT || t.kind == AT_TASK_PROLONG;
    if (t.reserved != 0 || (t.grid2 != nullptr && !two_level)) return "reserved task fields must be zero";
    const at_grid_s *g = task_grid(t);
    const bool needs_grid = t.kind == AT_TASK_ACTIVATE || t.kind == AT_TASK_LISTGEN || t.kind == AT_TASK_STENCIL ||
                            t.kind == AT_TASK_P2G || t.kind == AT_TASK_G2P || two_level || is_mpm_kind(t.kind);
    if (t.kind < AT_TASK_ACTIVATE || t.kind > AT_TASK_G2P_APIC) return "unknown task kind";
    if (needs_grid && !g) return "task needs a grid";
    auto chan_ok = [&](int c, int span) { return g && c >= 0 && c + span <= g->desc.channels; };
    switch (t.kind) {
    case AT_TASK_ACTIVATE:
        if (t.op != AT_COORD_VOXEL && t.op != AT_COORD_BLOCK) return "activate: bad coordinate kind";
        if (t.n < 0 || (t.n > 0 && !t.ext[0])) return "activate: bad coordinates";
        break;
    case AT_TASK_LISTGEN: break;
    case AT_TASK_STENCIL: {
        const int nc = op_nch(t.op);
        if (nc < 0) return "stencil: unknown op";
        if (t.op == AT_OP_FILL) {
            int cnt = 0;
            for (int q = 0; q < 7; ++q)
                if (t.ch[q] >= 0) {
                    if (!chan_ok(t.ch[q], 1)) return "fill: channel out of range";
                    ++cnt;
                }
            if (cnt == 0) return "fill: no channel";
            if (t.ch[7] >= 0) return "fill: at most 7 channels";
        } else if ((t.op == AT_OP_ADVECT || t.op == AT_OP_MACCORMACK) && t.param[1] != 0.f && t.param[1] != 1.f) {
            return "advect: param[1] (back-trace) must be 0 (Euler) or 1 (RK3)";
        } else if (t.op == AT_OP_ADVECT) {
            if (!chan_ok(t.ch[0], 1) || !chan_ok(t.ch[1], 3) || !chan_ok(t.ch[2], 1)) return "advect: channel out of range";
            if (t.ch[2] == t.ch[0] || (t.ch[2] >= t.ch[1] && t.ch[2] < t.ch[1] + 3))
                return "advect: the output aliases an input";
        } else if (t.op == AT_OP_MACCORMACK) {
            if (!chan_ok(t.ch[0], 1) || !chan_ok(t.ch[1], 3) || !chan_ok(t.ch[2], 1) || !chan_ok(t.ch[3], 1) ||
                !chan_ok(t.ch[4], 1))
                return "maccormack: channel out of range";
            const int o = t.ch[4];
            if (o == t.ch[0] || o == t.ch[2] || o == t.ch[3] || (o >= t.ch[1] && o < t.ch[1] + 3))
                return "maccormack: the output aliases an input";
        } else if (t.op == AT_OP_MPM_GRID) {
            if (!chan_ok(t.ch[0], 1) || !chan_ok(t.ch[1], 3) || !chan_ok(t.ch[2], 3)) return "mpm_grid: channel out of range";
            if ((t.ch[0] >= t.ch[2] && t.ch[0] < t.ch[2] + 3) || (t.ch[2] > t.ch[1] - 3 && t.ch[2] < t.ch[1] + 3))
                return "mpm_grid: the velocity channels overlap the mass or momentum channels";
            if (!(t.param[2] >= 0.f) || t.param[2] != (float)(int)t.param[2]) return "mpm_grid: bound must be a whole number >= 0";
        } else if (t.op == AT_OP_NORMALISE) {
            if (!chan_ok(t.ch[0], 1) || !chan_ok(t.ch[1], 3) || !chan_ok(t.ch[2], 3)) return "normalise: channel out of range";
            // v may replace mv in place (each component reads its own mv before writing);
            // any other overlap would make one component read another's result
            if ((t.ch[0] >= t.ch[2] && t.ch[0] < t.ch[2] + 3) || (t.ch[2] != t.ch[1] && t.ch[2] > t.ch[1] - 3 && t.ch[2] < t.ch[1] + 3))
                return "normalise: the velocity channels overlap the mass or part of the momentum channels";
        } else {
            for (int q = 0; q < nc; ++q)
                if (!chan_ok(t.ch[q], 1)) return "stencil: channel out of range";
        }
        if ((t.op == AT_OP_LAP_UPDATE && t.ch[0] == t.ch[1]) || (t.op == AT_OP_JACOBI && (t.ch[2] == t.ch[0] || t.ch[2] == t.ch[1])) ||
            (t.op == AT_OP_DIFFUSE && (t.ch[2] == t.ch[0] || t.ch[2] == t.ch[1])) ||
            (t.op == AT_OP_DIFFUSE_ADJ && (t.ch[3] == t.ch[0] || t.ch[3] == t.ch[1] || t.ch[3] == t.ch[2] ||
                                           t.ch[4] == t.ch[0] || t.ch[4] == t.ch[1] || t.ch[4] == t.ch[2] || t.ch[3] == t.ch[4])))
            return "stencil: an output channel aliases an input read at an offset";
        break;
    }
    case AT_TASK_ADVECT:
        if (t.n < 0 || (t.n > 0 && (!t.ext[0] || !t.ext[1]))) return "advect: bad arrays";
        break;
    case AT_TASK_P2G:
        if (t.n < 0 || (t.n > 0 && (!t.ext[0] || !t.ext[1] || !t.ext[2]))) return "p2g: bad arrays";
        if (!chan_ok(t.ch[0], 1) || !chan_ok(t.ch[1], 3)) return "p2g: channel out of range";
        if (!(t.param[0] > 0.f)) return "p2g: dx must be positive";
        if (t.op != AT_ACT_PER_NODE && t.op != AT_ACT_PER_BLOCK && t.op != AT_ACT_NONE)
            return "p2g: bad activation mode";
        break;
    case AT_TASK_G2P:
        if (t.n < 0 || (t.n > 0 && (!t.ext[0] || !t.ext[1]))) return "g2p: bad arrays";
        if (!chan_ok(t.ch[0], 3)) return "g2p: channel out of range";
        if (!(t.param[0] > 0.f)) return "g2p: dx must be positive";
        break;
    case AT_TASK_P2G_MLS:
        if (t.n < 0 || (t.n > 0 && (!t.ext[0] || !t.ext[1] || !t.ext[2] || !t.ext[3]))) return "p2g_mls: bad arrays";
        if (!chan_ok(t.ch[0], 1) || !chan_ok(t.ch[1], 3)) return "p2g_mls: channel out of range";
        if (!(t.param[0] > 0.f)) return "p2g_mls: dx must be positive";
        if (t.op != AT_ACT_PER_NODE && t.op != AT_ACT_PER_BLOCK && t.op != AT_ACT_NONE)
            return "p2g_mls: bad activation mode";
        break;
    case AT_TASK_G2P_APIC:
        if (t.n < 0 || (t.n > 0 && (!t.ext[0] || !t.ext[1] || !t.ext[2]))) return "g2p_apic: bad arrays";
        if (t.ext[1] == t.ext[2] || t.ext[0] == t.ext[1] || t.ext[0] == t.ext[2]) return "g2p_apic: arrays alias";
        if (!chan_ok(t.ch[0], 3)) return "g2p_apic: channel out of range";
        if (!(t.param[0] > 0.f)) return "g2p_apic: dx must be positive";
        break;
    case AT_TASK_RESTRICT:
    case AT_TASK_PROLONG: {
        const at_grid_s *c = reinterpret_cast<const at_grid_s *>(t.grid2);
        if (!c) return "two-level task needs the coarse grid in grid2";
        if (c == g) return "two-level task: the coarse grid must differ from the fine grid";
        if (c->desc.n[0] * 2 != g->desc.n[0] || c->virt != g->virt)
            return "two-level task: the coarse grid must have half the fine domain edge (and the same handle kind)";
        const int fch = t.kind == AT_TASK_RESTRICT ? t.ch[0] : t.ch[1];
        const int cch = t.kind == AT_TASK_RESTRICT ? t.ch[1] : t.ch[0];
        if (!chan_ok(fch, 1) || cch < 0 || cch >= c->desc.channels) return "two-level task: channel out of range";
        for (int q = 2; q < 8; ++q)
            if (t.ch[q] != -1) return "two-level task: unused channels must be -1";
        break;
    }
    }
    return "";
}

void derive(Node &nd, const at_task *tasks) {
    const at_task &t0 = tasks[nd.members[0].task];
    const at_grid_s *g = task_grid(t0);
    switch (t0.kind) {
    case AT_TASK_STENCIL:
    case AT_TASK_RESTRICT:
    case AT_TASK_PROLONG: nd.loop = LT_STRUCT; nd.loop_grid = g->uid; nd.range = 0; break;
    case AT_TASK_LISTGEN: nd.loop = LT_SERIAL; nd.loop_grid = 0; nd.range = 0; break;
    default: nd.loop = LT_RANGE; nd.loop_grid = 0; nd.range = t0.n; break;
    }
    nd.acc.clear();
    for (size_t m = 0; m < nd.members.size(); ++m)
        member_accesses(tasks[nd.members[m].task], nd.members[m], nd.check_activation, (int16_t)m, nd.acc);
    // A fused MLS-MPM node runs as one pass over the particles: what a member
    // produces at the loop index (the gather's v and C, stored or not, and the
    // advected x) reaches the later members in registers.  Their reads of
    // those arrays are internal to the node and leave its access list.
    bool mpm = false;
    for (const Member &mb : nd.members) mpm |= is_mpm_kind(tasks[mb.task].kind);
    if (!mpm || nd.members.size() < 2) return;
    std::vector<std::pair<StateKey, int>> produced;   // array, producing member
    for (size_t m = 0; m < nd.members.size(); ++m) {
        const at_task &t = tasks[nd.members[m].task];
        if (t.kind == AT_TASK_G2P_APIC) {
            produced.push_back({EXT(t.ext[1]), (int)m});
            produced.push_back({EXT(t.ext[2]), (int)m});
        } else if (t.kind == AT_TASK_ADVECT) {
            produced.push_back({EXT(t.ext[0]), (int)m});
        }
    }
    std::vector<Access> kept;
    kept.reserve(nd.acc.size());
    for (Access a : nd.acc) {
        if ((a.mode & M_R) && a.s.kind == ST_EXT && a.pattern == P_ELEM && (a.flags & F_UNIQUE)) {
            bool internal = false;
            for (const auto &pr : produced) internal |= pr.first == a.s && pr.second < a.member;
            if (internal) {
                a.mode &= (uint8_t)~M_R;
                if (!a.mode) continue;
            }
        }
        kept.push_back(a);
    }
    nd.acc.swap(kept);
}

uint64_t hash_window(const at_task *tasks, int n, uint32_t flags, int max_fuse) {
    uint64_t h = mix(0xa5a5ull, flags);
    h = mix(h, (uint64_t)max_fuse);
    h = mix(h, (uint64_t)n);
    for (int i = 0; i < n; ++i) {
        const at_task &t = tasks[i];
        const at_grid_s *g = task_grid(t);
        h = mix(h, (uint64_t)(uint32_t)t.kind | ((uint64_t)(uint32_t)t.op << 32));
        h = mix(h, t.flags);
        h = mix(h, g ? g->uid : 0);
        const at_grid_s *g2 = reinterpret_cast<const at_grid_s *>(t.grid2);
        h = mix(h, g2 ? g2->uid : 0);
        for (int q = 0; q < 8; ++q) h = mix(h, (uint64_t)(uint32_t)t.ch[q]);
        for (int q = 0; q < 8; ++q) {
            uint32_t b;
            std::memcpy(&b, &t.param[q], 4);
            h = mix(h, b);
        }
        for (int q = 0; q < 4; ++q) h = mix(h, (uint64_t)(uintptr_t)t.ext[q]);
        h = mix(h, (uint64_t)t.n);
    }
    return h;
}

// ------------------------------------------------------------------ planner

Planner::Planner(const at_task *tasks, int n, uint32_t flags, int max_fuse, bool batch_fusions)
    : tasks_(tasks), n_(n), flags_(flags), max_fuse_(max_fuse < 1 ? 1 : max_fuse), batch_(batch_fusions) {}

void Planner::build_eager() {
    nodes.clear();
    nodes.reserve(n_);
    for (int i = 0; i < n_; ++i) {
        Node nd;
        nd.members.push_back({i, ~0u});
        nd.check_activation = true;
        nd.act_mode = is_scatter_kind(tasks_[i].kind) ? tasks_[i].op : AT_ACT_PER_NODE;
        derive(nd, tasks_);
        nodes.push_back(std::move(nd));
    }
}

// Activation demotion (Section 6.3).  (a) A struct-for only ever writes at
// its loop index, i.e. inside blocks of the list it iterates, which are
// active: the activation check of those writes can never activate anything
// and is dropped, so the task no longer modifies the mask.  (b) An
// activation identical to one already performed (same grid, coordinate
// array at the same version, same count), with no deactivation of the mask
// since, activates nothing and is removed.  (c) Particle scatter activates
// data-dependent nodes; its 27 per-node checks are coarsened to one
// activation per distinct touched block (the same blocks become active).
bool Planner::pass_ad(const Persist &start) {
    bool changed = false;
    for (Node &nd : nodes) {
        // a struct-for writing its own grid at the loop index only touches
        // listed (active) blocks; a restriction writes another grid and is
        // demoted by its signature below
        if (nd.loop == LT_STRUCT && nd.check_activation && !node_has_kind(nd, tasks_, AT_TASK_RESTRICT)) {
            nd.check_activation = false;
            counters.activations_demoted += (int64_t)nd.members.size();
            derive(nd, tasks_);
            changed = true;
        }
        if (nd.act_mode == AT_ACT_PER_NODE &&
            (node_has_kind(nd, tasks_, AT_TASK_P2G) || node_has_kind(nd, tasks_, AT_TASK_P2G_MLS))) {
            nd.act_mode = AT_ACT_PER_BLOCK;
            counters.activations_demoted += 1;
            changed = true;
        }
    }
    Sim S = simulate(nodes, tasks_, start);
    std::unordered_map<uint64_t, std::unordered_set<uint64_t>> sigs;
    std::vector<Node> kept;
    kept.reserve(nodes.size());
    for (int i = 0; i < S.n; ++i) {
        const at_task &t0 = tasks_[nodes[i].members[0].task];
        if (t0.kind == AT_TASK_ACTIVATE) {
            const uint64_t gu = task_grid(t0)->uid;
            auto it = sigs.find(gu);
            if (it == sigs.end()) {
                auto st = start.act_sigs.find(gu);
                it = sigs.emplace(gu, st == start.act_sigs.end() ? std::unordered_set<uint64_t>() : st->second).first;
            }
            if (it->second.count(S.act_sig[i])) {
                counters.activations_demoted += 1;
                changed = true;
                continue;
            }
            it->second.insert(S.act_sig[i]);
        }
        if (t0.kind == AT_TASK_RESTRICT && nodes[i].check_activation) {
            // the same list version of the fine grid was already restricted
            // into this coarse grid: every parent block is active
            const uint64_t cu = reinterpret_cast<const at_grid_s *>(t0.grid2)->uid;
            auto it = sigs.find(cu);
            if (it == sigs.end()) {
                auto st = start.act_sigs.find(cu);
                it = sigs.emplace(cu, st == start.act_sigs.end() ? std::unordered_set<uint64_t>() : st->second).first;
            }
            if (it->second.count(S.act_sig[i])) {
                nodes[i].check_activation = false;
                derive(nodes[i], tasks_);
                counters.activations_demoted += 1;
                changed = true;
            } else {
                it->second.insert(S.act_sig[i]);
            }
        }
        kept.push_back(std::move(nodes[i]));
    }
    nodes.swap(kept);
    return changed;
}

// List generation removal (Section 6.2): list generation is idempotent in
// its inputs, so a listgen whose mask state has the version the current list
// was generated from is removed; its consumers read the existing list.
bool Planner::pass_lgr(const Persist &start) {
    bool changed = false;
    std::unordered_map<uint64_t, uint64_t> maskv, lsrc;
    auto get_mask = [&](uint64_t g) -> uint64_t & {
        auto it = maskv.find(g);
        if (it == maskv.end()) it = maskv.emplace(g, start.ver(MASK(g))).first;
        return it->second;
    };
    auto get_src = [&](uint64_t g) -> uint64_t & {
        auto it = lsrc.find(g);
        if (it == lsrc.end()) {
            auto st = start.list_src.find(g);
            it = lsrc.emplace(g, st == start.list_src.end() ? ~0ull : st->second).first;
        }
        return it->second;
    };
    std::vector<Node> kept;
    kept.reserve(nodes.size());
    std::vector<uint64_t> bumped;
    for (Node &nd : nodes) {
        const at_task &t0 = tasks_[nd.members[0].task];
        if (t0.kind == AT_TASK_LISTGEN) {
            const uint64_t gu = task_grid(t0)->uid;
            if (get_src(gu) == get_mask(gu)) {
                counters.listgens_removed += 1;
                changed = true;
                continue;
            }
            get_src(gu) = get_mask(gu);
        }
        bumped.clear();
        for (const Access &a : nd.acc)
            if ((a.mode & M_W) && a.s.kind == ST_MASK &&
                std::find(bumped.begin(), bumped.end(), a.s.obj) == bumped.end()) {
                bumped.push_back(a.s.obj);
                get_mask(a.s.obj) += 1;
            }
        kept.push_back(std::move(nd));
    }
    nodes.swap(kept);
    return changed;
}

// Dead store elimination (Section 6.5).  A store of member task A to a value
// (or external) state S is dead when the next access to S in the window is a
// write by a task B that does not read S, overwrites it completely, and
// covers A's loop domain: B a struct-for over the same grid and a list at
// least as new (masks only grow inside a window), or B a range-for of the
// same length over arrays indexed uniquely at the loop index.  Reads of S in
// between (including stencil and gather reads) keep it alive, and so does
// the end of the window (the host may observe S).  A task whose stores are
// all dead is removed; FILL and NORMALISE drop single channels.
bool Planner::pass_dse(const Persist &start) {
    Sim S = simulate(nodes, tasks_, start);
    struct Op {
        int node, member;
        bool activating;
        std::vector<Access> acc;
    };
    std::vector<Op> ops;
    for (int i = 0; i < (int)nodes.size(); ++i) {
        const Node &nd = nodes[i];
        for (int m = 0; m < (int)nd.members.size(); ++m) {
            Op op{i, m, false, {}};
            for (const Access &a : nd.acc)
                if (a.member == m) {
                    op.acc.push_back(a);
                    if (a.flags & F_ACTIVATING) op.activating = true;
                }
            ops.push_back(std::move(op));
        }
    }
    auto covers = [&](const Op &b, const Op &a, const Access &wb, const Access &wa) {
        const Node &na = nodes[a.node], &nb = nodes[b.node];
        if (na.loop == LT_STRUCT && nb.loop == LT_STRUCT)
            return na.loop_grid == nb.loop_grid && S.list_ver[b.node] >= S.list_ver[a.node];
        if (na.loop == LT_RANGE && nb.loop == LT_RANGE)
            return na.range == nb.range && wa.s.kind == ST_EXT && (wa.flags & F_UNIQUE) && (wb.flags & F_UNIQUE);
        return false;
    };
    // dead[(op, state)]
    std::vector<std::vector<StateKey>> dead(ops.size());
    int64_t ndead = 0;
    for (size_t p = 0; p < ops.size(); ++p) {
        if (ops[p].activating) continue;
        for (const Access &w : ops[p].acc) {
            if (!(w.mode & M_W) || (w.s.kind != ST_VALUE && w.s.kind != ST_EXT)) continue;
            bool is_dead = false;
            for (size_t q = p + 1; q < ops.size(); ++q) {
                bool rd = false, wrt = false, ok = true;
                const Access *wq = nullptr;
                for (const Access &a : ops[q].acc) {
                    if (!(a.s == w.s)) continue;
                    if (a.mode & M_R) rd = true;
                    if (a.mode & M_W) {
                        wrt = true;
                        wq = &a;
                        if (!(a.flags & F_FULL)) ok = false;
                    }
                }
                if (!rd && !wrt) continue;
                is_dead = !rd && wrt && ok && covers(ops[q], ops[p], *wq, w);
                break;
            }
            if (is_dead) {
                dead[p].push_back(w.s);
                ++ndead;
            }
        }
    }
    if (ndead == 0) return false;
    bool changed = false;
    for (size_t p = 0; p < ops.size(); ++p) {
        if (dead[p].empty()) continue;
        Node &nd = nodes[ops[p].node];
        Member &mb = nd.members[ops[p].member];
        const at_task &t = tasks_[mb.task];
        auto is_dead_ch = [&](int ch) {
            for (const StateKey &s : dead[p])
                if (s.kind == ST_VALUE && s.ch == ch) return true;
            return false;
        };
        if (t.kind == AT_TASK_STENCIL && t.op == AT_OP_FILL) {
            for (int q = 0; q < 7; ++q)
                if (t.ch[q] >= 0 && ((mb.keep >> q) & 1u) && is_dead_ch(t.ch[q])) {
                    mb.keep &= ~(1u << q);
                    counters.stores_eliminated += 1;
                    changed = true;
                }
            bool any = false;
            for (int q = 0; q < 7; ++q) any |= t.ch[q] >= 0 && ((mb.keep >> q) & 1u);
            if (!any) mb.task = -1;
        } else if (t.kind == AT_TASK_G2P_APIC) {
            // the stores of v (keep bit 0) and C (bit 1) are dropped one by
            // one; the gather stays while a later member of its node uses
            // its results in registers
            for (int q = 0; q < 2; ++q) {
                const StateKey sk = EXT(t.ext[1 + q]);
                if (((mb.keep >> q) & 1u) && std::find(dead[p].begin(), dead[p].end(), sk) != dead[p].end()) {
                    mb.keep &= ~(1u << q);
                    counters.stores_eliminated += 1;
                    changed = true;
                }
            }
            if ((mb.keep & 3u) == 0 && ops[p].member == (int)nd.members.size() - 1) mb.task = -1;
        } else if (t.kind == AT_TASK_STENCIL && t.op == AT_OP_NORMALISE) {
            for (int q = 0; q < 3; ++q)
                if (((mb.keep >> q) & 1u) && is_dead_ch(t.ch[2] + q)) {
                    mb.keep &= ~(1u << q);
                    counters.stores_eliminated += 1;
                    changed = true;
                }
            if ((mb.keep & 7u) == 0) mb.task = -1;
        } else {
            // every store of the member must be dead to drop it
            int nw = 0;
            for (const Access &a : ops[p].acc)
                if ((a.mode & M_W) && (a.s.kind == ST_VALUE || a.s.kind == ST_EXT)) ++nw;
            if (nw > 0 && nw == (int)dead[p].size()) {
                counters.stores_eliminated += nw;
                mb.task = -1;
                changed = true;
            }
        }
    }
    if (!changed) return false;
    std::vector<Node> kept;
    for (Node &nd : nodes) {
        std::vector<Member> ms;
        for (const Member &m : nd.members)
            if (m.task >= 0) ms.push_back(m);
        if (ms.empty()) continue;
        nd.members.swap(ms);
        derive(nd, tasks_);
        kept.push_back(std::move(nd));
    }
    nodes.swap(kept);
    return true;
}

namespace {

// A fused task must map onto a pre-built kernel composition: any chain of
// struct-for ops over one grid (run per voxel in program order), or
// gather -> advect -> scatter over the same particle arrays.
bool executable_pair(const Node &A, const Node &B, const at_task *tasks) {
    if (A.loop == LT_STRUCT) {
        if (A.check_activation != B.check_activation) return false;
        if (A.members.size() + B.members.size() > (size_t)kMaxOps) return false;
        for (const Node *N : {&A, &B})
            for (const Member &m : N->members)
                if (tasks[m.task].kind != AT_TASK_STENCIL) return false;
        return true;
    }
    if (A.loop == LT_RANGE) {
        // PIC members (G2P, P2G) and MLS-MPM members (G2P_APIC, P2G_MLS,
        // sharing C as well) do not mix; ADVECT joins either
        int rank_prev = -1, family = 0;
        const void *x = nullptr, *v = nullptr, *C = nullptr;
        for (const Node *N : {&A, &B})
            for (const Member &m : N->members) {
                const at_task &t = tasks[m.task];
                if (!is_particle_kind(t.kind) || !(t.flags & AT_TASKF_LOOP_UNIQUE)) return false;
                const int rank = (t.kind == AT_TASK_G2P || t.kind == AT_TASK_G2P_APIC) ? 0
                               : t.kind == AT_TASK_ADVECT ? 1 : 2;
                if (rank <= rank_prev) return false;
                rank_prev = rank;
                if (t.kind != AT_TASK_ADVECT) {
                    const int fam = is_mpm_kind(t.kind) ? 2 : 1;
                    if (family && fam != family) return false;
                    family = fam;
                }
                const void *tx = t.ext[0], *tv = t.ext[1];
                if ((x && tx != x) || (v && tv != v)) return false;
                x = tx;
                v = tv;
                if (is_mpm_kind(t.kind)) {
                    if (C && t.ext[2] != C) return false;
                    C = t.ext[2];
                }
            }
        return true;
    }
    return false;
}

}  // namespace

// One greedy round of task fusion (Section 6.4; supplement Section 2).
// A and B (A before B) are fused when (1) there is no path of length >= 2
// between them, checked with the transitive closure; (2) both are struct-fors
// over the same grid and the same list version, or range-fors of the same
// length; (3) every state they share with a write is accessed element-wise at
// the loop index, uniquely per iteration, in both; (4) neither was fused more
// than max_fuse_per_task times this round.  Fusions are applied one at a
// time; after each the graph is rebuilt from a topological order of the
// contracted graph.
// Fusion in greedy order: the first fusible pair (a, b) of the current graph
// (smallest a, then smallest b) is contracted, and the search starts again.
// One simulation serves several contractions when the result provably equals
// that one-at-a-time order: after picking (a1, b1), a node strictly between
// them with any fusible partner ends the batch (only the contracted graph can
// tell whether it still fuses), while a pair (a2, b2) with a2 > b1 is the one
// the contracted graph would pick next -- contracting (a1, b1) adds paths
// only through the merged node, which no path starting after b1 can reach,
// and leaves every other node's accesses, list version and fusion count as
// they were.  Pairs picked this way have disjoint, ordered spans, so
// contracting them together keeps the graph acyclic.  The nodes before the
// batch's first pair had no fusible partner and keep their places (the
// re-sort breaks ties in the old order), so the next search resumes there.
// With more than one fusion per task and round, a merged node may fuse
// again, so the batch holds one pair and every search starts at the front.
bool Planner::pass_fuse_round(const Persist &start) {
    std::vector<int> fused(nodes.size(), 0);
    bool any = false;
    int from = 0;
    for (;;) {
        Sim S = simulate(nodes, tasks_, start);
        std::vector<uint64_t> reach = closure(S);
        auto fusible = [&](int a, int b) {
            const Node &A = nodes[a], &B = nodes[b];
            if (B.loop != A.loop) return false;
            if (A.loop == LT_STRUCT && (A.loop_grid != B.loop_grid || S.list_ver[a] != S.list_ver[b])) return false;
            if (A.loop == LT_RANGE && A.range != B.range) return false;
            if (!executable_pair(A, B, tasks_)) return false;
            // criterion 1
            if (S.edge(a, b)) {
                for (int c = a + 1; c < b; ++c)
                    if (bit(reach, S.words, a, c) && bit(reach, S.words, c, b)) return false;
            } else if (bit(reach, S.words, a, b)) {
                return false;
            }
            // criterion 3
            for (const Access &x : A.acc)
                for (const Access &y : B.acc) {
                    if (!(x.s == y.s) || !((x.mode | y.mode) & M_W)) continue;
                    if (x.pattern != P_ELEM || y.pattern != P_ELEM || !(x.flags & F_UNIQUE) || !(y.flags & F_UNIQUE))
                        return false;
                }
            return true;
        };
        std::vector<std::pair<int, int>> batch;
        std::vector<char> taken(S.n, 0);
        int span_hi = -1;
        for (int a = from; a < S.n; ++a) {
            if (taken[a] || fused[a] >= max_fuse_ || nodes[a].loop == LT_SERIAL) continue;
            int pick = -1;
            for (int b = a + 1; b < S.n && pick < 0; ++b)
                if (!taken[b] && fused[b] < max_fuse_ && fusible(a, b)) pick = b;
            if (pick < 0) continue;
            if (a < span_hi) break;
            batch.push_back({a, pick});
            taken[a] = taken[pick] = 1;
            span_hi = pick;
            if (max_fuse_ != 1 || !batch_) break;
        }
        if (batch.empty()) break;
        if (max_fuse_ == 1 && batch_) from = batch.front().first;
        // contract every pair (b into a), then re-sort topologically, ties
        // in the old order
        std::vector<int> into(S.n, -1);
        for (const auto &pr : batch) into[pr.second] = pr.first;
        const int nn = S.n - (int)batch.size();
        std::vector<int> newid(S.n);
        std::vector<Node> pool;
        std::vector<int> key, fcnt;
        pool.reserve(nn);
        std::vector<int> partner(S.n, -1);
        for (const auto &pr : batch) partner[pr.first] = pr.second;
        for (int i = 0; i < S.n; ++i) {
            if (into[i] >= 0) continue;
            newid[i] = (int)pool.size();
            if (partner[i] >= 0) {
                const int fb = partner[i];
                Node AB = nodes[i];
                for (const Member &m : nodes[fb].members) AB.members.push_back(m);
                if (node_has_kind(nodes[fb], tasks_, AT_TASK_P2G) || node_has_kind(nodes[fb], tasks_, AT_TASK_P2G_MLS))
                    AB.act_mode = nodes[fb].act_mode;
                derive(AB, tasks_);
                pool.push_back(std::move(AB));
                fcnt.push_back(std::max(fused[i], fused[fb]) + 1);
            } else {
                pool.push_back(std::move(nodes[i]));
                fcnt.push_back(fused[i]);
            }
            key.push_back(i);
        }
        for (int i = 0; i < S.n; ++i)
            if (into[i] >= 0) newid[i] = newid[into[i]];
        std::vector<std::vector<int>> succ(nn);
        std::vector<int> indeg(nn, 0);
        for (int i = 0; i < S.n; ++i)
            for (int w = 0; w < S.words; ++w) {
                uint64_t bits = S.adj[(size_t)i * S.words + w];
                while (bits) {
                    const int j = w * 64 + __builtin_ctzll(bits);
                    bits &= bits - 1;
                    const int u = newid[i], v = newid[j];
                    if (u == v) continue;
                    if (std::find(succ[u].begin(), succ[u].end(), v) == succ[u].end()) {
                        succ[u].push_back(v);
                        indeg[v] += 1;
                    }
                }
            }
        std::priority_queue<std::pair<int, int>, std::vector<std::pair<int, int>>, std::greater<>> ready;
        for (int u = 0; u < nn; ++u)
            if (indeg[u] == 0) ready.push({key[u], u});
        std::vector<Node> order;
        std::vector<int> ofused;
        order.reserve(nn);
        while (!ready.empty()) {
            const int u = ready.top().second;
            ready.pop();
            order.push_back(std::move(pool[u]));
            ofused.push_back(fcnt[u]);
            for (int v : succ[u])
                if (--indeg[v] == 0) ready.push({key[v], v});
        }
        // criterion 1 and the ordered spans guarantee the contracted graph is acyclic
        nodes.swap(order);
        fused.swap(ofused);
        counters.fusions += (int64_t)batch.size();
        any = true;
    }
    return any;
}

void Planner::optimize(const Persist &start) {
    for (int iter = 0; iter < 64; ++iter) {
        bool changed = false;
        if (flags_ & AT_OPT_AD) changed |= pass_ad(start);
        if (flags_ & AT_OPT_LGR) changed |= pass_lgr(start);
        if (flags_ & AT_OPT_DSE) changed |= pass_dse(start);
        if (flags_ & AT_OPT_FUSE) changed |= pass_fuse_round(start);
        if (!changed) break;
    }
}

std::vector<uint8_t> neighbour_tables_valid(const std::vector<Node> &nodes, const at_task *tasks, const Persist &P) {
    std::vector<uint8_t> ok(nodes.size(), 0);
    std::unordered_map<uint64_t, uint64_t> maskv, lsrc;
    auto mv = [&](uint64_t g) -> uint64_t & {
        auto it = maskv.find(g);
        if (it == maskv.end()) it = maskv.emplace(g, P.ver(MASK(g))).first;
        return it->second;
    };
    auto ls = [&](uint64_t g) -> uint64_t & {
        auto it = lsrc.find(g);
        if (it == lsrc.end()) {
            auto st = P.list_src.find(g);
            it = lsrc.emplace(g, st == P.list_src.end() ? ~0ull : st->second).first;
        }
        return it->second;
    };
    std::vector<uint64_t> bumped;
    for (size_t i = 0; i < nodes.size(); ++i) {
        const Node &nd = nodes[i];
        const at_task &t0 = tasks[nd.members[0].task];
        if (nd.loop == LT_STRUCT) ok[i] = ls(nd.loop_grid) == mv(nd.loop_grid);
        if (t0.kind == AT_TASK_LISTGEN) {
            const uint64_t g = task_grid(t0)->uid;
            ls(g) = mv(g);
        }
        bumped.clear();
        for (const Access &a : nd.acc)
            if ((a.mode & M_W) && a.s.kind == ST_MASK &&
                std::find(bumped.begin(), bumped.end(), a.s.obj) == bumped.end()) {
                bumped.push_back(a.s.obj);
                mv(a.s.obj) += 1;
            }
    }
    return ok;
}

void Planner::commit(const std::vector<Node> &nodes, const at_task *tasks, Persist &p) {
    Sim S = simulate(nodes, tasks, p);
    for (int i = 0; i < S.n; ++i) {
        const at_task &t0 = tasks[nodes[i].members[0].task];
        if (t0.kind == AT_TASK_LISTGEN) p.list_src[task_grid(t0)->uid] = S.mask_at[i];
        if (t0.kind == AT_TASK_ACTIVATE) p.act_sigs[task_grid(t0)->uid].insert(S.act_sig[i]);
        if (t0.kind == AT_TASK_RESTRICT)
            p.act_sigs[reinterpret_cast<const at_grid_s *>(t0.grid2)->uid].insert(S.act_sig[i]);
    }
    for (const auto &kv : S.cur) p.version[kv.first] = kv.second;
}

std::vector<uint8_t> Planner::fingerprint(const at_task *tasks, int n, const Persist &p) {
    std::vector<uint8_t> fp;
    std::unordered_map<uint64_t, int> seen;
    std::unordered_map<uint64_t, uint64_t> extv;
    for (int i = 0; i < n; ++i) {
        const at_task &t = tasks[i];
        const at_grid_s *g = task_grid(t);
        if (g && !seen.count(g->uid)) {
            seen[g->uid] = 1;
            auto it = p.list_src.find(g->uid);
            fp.push_back(it != p.list_src.end() && it->second == p.ver(MASK(g->uid)));
        }
        if (t.kind == AT_TASK_ACTIVATE) {
            const uint64_t key = (uint64_t)(uintptr_t)t.ext[0];
            auto ev = extv.find(key);
            const uint64_t ver = ev != extv.end() ? ev->second : p.ver(EXT(t.ext[0]));
            auto it = p.act_sigs.find(g->uid);
            fp.push_back(it != p.act_sigs.end() && it->second.count(activation_sig(t, ver)));
        }
        if (t.kind == AT_TASK_RESTRICT) {
            // only the list version at the window's start can match a known
            // signature: versions made inside the window are new
            const at_grid_s *c = reinterpret_cast<const at_grid_s *>(t.grid2);
            auto it = p.act_sigs.find(c->uid);
            fp.push_back(it != p.act_sigs.end() && it->second.count(restrict_sig(t, p.ver(LIST(g->uid)))));
            if (!seen.count(c->uid)) {
                seen[c->uid] = 1;
                auto ls = p.list_src.find(c->uid);
                fp.push_back(ls != p.list_src.end() && ls->second == p.ver(MASK(c->uid)));
            }
        }
        // external arrays written inside the window
        if (t.kind == AT_TASK_ADVECT) {
            const uint64_t key = (uint64_t)(uintptr_t)t.ext[0];
            auto ev = extv.find(key);
            extv[key] = (ev != extv.end() ? ev->second : p.ver(EXT(t.ext[0]))) + 1;
        }
        if (t.kind == AT_TASK_G2P || t.kind == AT_TASK_G2P_APIC) {
            const uint64_t key = (uint64_t)(uintptr_t)t.ext[1];
            auto ev = extv.find(key);
            extv[key] = (ev != extv.end() ? ev->second : p.ver(EXT(t.ext[1]))) + 1;
        }
        if (t.kind == AT_TASK_G2P_APIC || t.kind == AT_TASK_P2G_MLS) {
            void *w = t.kind == AT_TASK_G2P_APIC ? t.ext[2] : t.ext[3];
            const uint64_t key = (uint64_t)(uintptr_t)w;
            auto ev = extv.find(key);
            extv[key] = (ev != extv.end() ? ev->second : p.ver(EXT(w))) + 1;
        }
    }
    return fp;
}

}  // namespace ats
