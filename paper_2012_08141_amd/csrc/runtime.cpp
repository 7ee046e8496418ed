// Grid runtime, execution engine and the C ABI of libatsparse.
//
// The engine follows the paper's asynchronous execution engine (Section 7.1):
// tasks of a window (one at_run_sequence call, or everything queued by
// at_enqueue until a flush) are planned together -- state-flow graph plus the
// passes selected by the caller -- and launched in order on the caller's
// stream with no host synchronisation.  After each window only the
// information carried by the latest owners of each state is kept (partial
// SFG garbage collection), and optimized plans are cached under a hash of the
// window's task descriptors (the IR-bank analogue of Section 7.2).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"
#include "sfg.hpp"

using namespace ats;

namespace {

thread_local std::string g_err;

at_status fail(at_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

at_status hip_fail(hipError_t e, const char *what) {
    return fail(AT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

struct CacheEntry {
    std::vector<uint8_t> fp;
    std::vector<Node> nodes;
    PlanCounters counters;
};

// A flushed window on its way through the asynchronous pipeline
// (AT_OPTION_ASYNC): the optimizer thread fills in the plan, the launcher
// thread launches it.
struct PendingWindow {
    std::vector<at_task> tasks;
    uint32_t flags = 0;
    hipStream_t stream = nullptr;
    int device = -1;
    bool any_virt = false;
    std::vector<Node> nodes;
    std::vector<uint8_t> tables;
    PlanCounters ctr{};
    int64_t hits = 0;
    double us = 0;
};

struct AsyncPipe {
    std::mutex mu;
    std::condition_variable cv;      // work arrived, or a worker finished some
    std::deque<std::unique_ptr<PendingWindow>> to_plan, to_launch;
    int busy = 0;                    // windows a worker has taken and not finished
    at_status err = AT_OK;           // first failure since it was last reported
    std::string msg;
    at_stats sum{};                  // counters of the windows launched since the last sync
    std::thread optimizer, launcher;
};

struct Engine {
    std::recursive_mutex mu;
    bool async = false;                  // flushes go to the pipeline (AT_OPTION_ASYNC)
    bool verify_demoted = false;         // AT_OPTION_VERIFY_DEMOTED
    std::unique_ptr<AsyncPipe> pipe;     // started when async is first switched on
    Persist persist;
    std::unordered_map<uint64_t, CacheEntry> cache;
    int max_fuse = 1;
    int64_t flush_period = 0;
    uint32_t opt_flags = AT_OPT_ALL;
    bool plan_cache = true;
    bool g2p_bins = true;   // gathers may use the source grid's bins
    int32_t bin_reuse = 8;  // scatters that may reuse a binning before the particles are binned again
    bool fuse_batch = true; // one graph simulation may serve several fusions (same plans)
    bool static_ws = false; // the scatter being run bins through the static workspace (at_p2g_static)
    std::unordered_map<uint64_t, at_grid_s *> live;   // device grids by uid
    // Inside one window only its own nodes touch external arrays, so a
    // binned scatter's particle records still hold the current positions
    // when the same window has not advected those positions since.
    uint64_t window_seq = 0;                                // bumped per executed window
    std::unordered_map<const void *, int64_t> pos_writes;   // advections per position array, this window
    std::vector<at_task> queue;
    hipStream_t queue_stream = nullptr;
    std::atomic<int64_t> dispatches{0};
    uint64_t next_uid = 1;
    // per-launch timing (at_timing_enable)
    struct Timed {
        int32_t kind, op, members;
        hipEvent_t a, b;
    };
    bool timing = false;
    std::vector<hipEvent_t> ev_free;
    std::vector<Timed> timed;
    // HIP graphs of repeated optimized windows (see run_window)
    struct Graph {
        hipGraphExec_t exec;
        int64_t dispatches;
        std::vector<uint64_t> uids;   // grids whose memory the launches use
    };
    bool graphs = false;
    std::unordered_map<uint64_t, Graph> graph_cache;
    hipStream_t capture_stream = nullptr;
};

Engine &E() {
    static Engine *e = new Engine();
    return *e;
}

at_grid_s *live_grid(uint64_t uid) {
    Engine &en = E();
    const auto it = en.live.find(uid);
    return it == en.live.end() ? nullptr : it->second;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t hdr, scan, bits, ptr, list, pcount, poff, pbins, pkr, pstage, pout, chan, total;
    int64_t pcap;
    int64_t ncells;
    int32_t cap, list_cap, R;
};

at_status layout_of(const at_grid_desc *d, Layout &L) {
    if (!d) return fail(AT_E_INVALID, "null grid description");
    if (d->n[0] <= 0 || d->n[0] % kBS != 0) return fail(AT_E_INVALID, "domain edge must be a positive multiple of 8");
    if (d->n[1] != d->n[0] || d->n[2] != d->n[0])
        return fail(AT_E_UNSUPPORTED, "only cubic domains are supported (n[0] == n[1] == n[2])");
    const int64_t R = d->n[0] / kBS;
    if (R > 1024) return fail(AT_E_INVALID, "domain edge above 8192 voxels");
    if (d->root_kind != AT_ROOT_BITMASK && d->root_kind != AT_ROOT_POINTER) return fail(AT_E_INVALID, "unknown root kind");
    if (d->channels < 1 || d->channels > 64) return fail(AT_E_INVALID, "channels must be in 1..64");
    L.R = (int32_t)R;
    L.ncells = R * R * R;
    if (d->root_kind == AT_ROOT_BITMASK) {
        L.cap = (int32_t)L.ncells;
    } else {
        if (d->capacity_blocks < 1 || d->capacity_blocks > L.ncells)
            return fail(AT_E_INVALID, "pointer root: capacity_blocks must be in 1..R^3");
        L.cap = d->capacity_blocks;
    }
    L.list_cap = (int32_t)(L.cap < L.ncells ? L.cap : L.ncells);
    size_t off = 0;
    L.hdr = off; off += 256;
    L.scan = off; off += kScanFlags * sizeof(uint64_t);
    L.bits = off; off += align256(((L.ncells + 31) / 32) * 4);
    L.ptr = off; if (d->root_kind == AT_ROOT_POINTER) off += align256(L.ncells * 4);
    L.list = off; off += align256((size_t)L.list_cap * kRec * sizeof(int32_t));
    if (d->particle_capacity < 0) return fail(AT_E_INVALID, "particle_capacity must be >= 0");
    L.pcap = d->particle_capacity;
    const size_t nc = (size_t)L.ncells;
    L.pcount = off; if (L.pcap) off += align256(nc * sizeof(int32_t));
    L.poff = off;   if (L.pcap) off += align256(nc * sizeof(int32_t));
    L.pbins = off;  if (L.pcap) off += align256(nc * 4 * sizeof(int32_t));
    L.pkr = off;    if (L.pcap) off += align256((size_t)L.pcap * 2 * sizeof(int32_t));
    L.pstage = off; if (L.pcap) off += align256((size_t)L.pcap * 8 * sizeof(float));
    L.pout = off;   if (L.pcap) off += align256((size_t)L.pcap * sizeof(int32_t));
    L.chan = off; off += (size_t)d->channels * L.cap * kBV * sizeof(float);
    L.total = off;
    return AT_OK;
}

at_status check_grid(at_grid g, bool need_device) {
    if (!g) return fail(AT_E_INVALID, "null grid handle");
    if (need_device && g->virt) return fail(AT_E_STATE, "planning handle has no device memory");
    return AT_OK;
}

// ------------------------------------------------------------ execution

int64_t dispatches_of(const Node &) { return 1; }

at_status execute_node(const Node &nd, const at_task *tasks, bool table, hipStream_t s) {
    const at_task &t0 = tasks[nd.members[0].task];
    const at_grid_s *g = task_grid(t0);
    // planning handles launch nothing
    for (const Member &m : nd.members) {
        const at_grid_s *gm = task_grid(tasks[m.task]);
        if (gm && gm->virt) return AT_OK;
    }
    hipError_t e = hipSuccess;
    switch (t0.kind) {
    case AT_TASK_ACTIVATE:
        e = launch_activate(g->dev, (const int32_t *)t0.ext[0], t0.n, t0.op, s);
        break;
    case AT_TASK_LISTGEN: {
        at_grid_s *gm = const_cast<at_grid_s *>(g);
        if (++gm->listgen_epoch == 0) gm->listgen_epoch = 1;
        e = launch_listgen(g->dev, g->dev.scan, gm->listgen_epoch, s);
        break;
    }
    case AT_TASK_STENCIL: {
        const Member &m0 = nd.members[0];
        const bool tiled = t0.op == AT_OP_LAP_UPDATE || t0.op == AT_OP_JACOBI || t0.op == AT_OP_DIFFUSE ||
                           t0.op == AT_OP_DIFFUSE_ADJ;
        bool tail = nd.members.size() > 1 && tiled && t0.op != AT_OP_DIFFUSE_ADJ && m0.keep == ~0u &&
                    !nd.check_activation && table && struct_for_kernel() == 0 &&
                    nd.members.size() - 1 <= (size_t)kMaxOps;
        for (size_t q = 1; tail && q < nd.members.size(); ++q) tail = tail_op_supported(tasks[nd.members[q].task].op);
        // verification of demoted writes runs every such node in the interpreter
        const bool verify = E().verify_demoted && !nd.check_activation;
        if (verify) tail = false;
        if (nd.members.size() == 1 && tiled && m0.keep == ~0u && !verify) {
            e = launch_stencil(g->dev, t0.op, t0.ch, t0.param[0], nd.check_activation ? 1 : 0, table ? 1 : 0, s);
        } else if (tail) {
            MicroProg prog{};
            prog.nops = (int32_t)nd.members.size() - 1;
            for (size_t q = 1; q < nd.members.size(); ++q) {
                const at_task &t = tasks[nd.members[q].task];
                MicroOp &op = prog.ops[q - 1];
                op.op = t.op;
                for (int c = 0; c < 7; ++c) op.ch[c] = t.ch[c];
                op.p = t.param[0];
                op.keep = nd.members[q].keep;
                op.p1 = t.param[1];
                op.p2 = t.param[2];
            }
            e = launch_stencil_tail(g->dev, t0.op, t0.ch, t0.param[0], prog, s);
        } else {
            MicroProg prog{};
            prog.nops = (int32_t)nd.members.size();
            prog.check = nd.check_activation ? 1 : 0;
            prog.table = table ? 1 : 0;
            prog.verify = verify ? 1 : 0;
            for (size_t q = 0; q < nd.members.size(); ++q) {
                const at_task &t = tasks[nd.members[q].task];
                MicroOp &op = prog.ops[q];
                op.op = t.op;
                for (int c = 0; c < 7; ++c) op.ch[c] = t.ch[c];
                op.p = t.param[0];
                op.keep = nd.members[q].keep;
                op.p1 = t.param[1];
                op.p2 = t.param[2];
            }
            if (verify || !variant_launch(g->dev, prog, s, e)) e = launch_micro(g->dev, prog, s);
        }
        break;
    }
    case AT_TASK_RESTRICT:
    case AT_TASK_PROLONG: {
        const at_grid_s *c = reinterpret_cast<const at_grid_s *>(t0.grid2);
        const bool r = t0.kind == AT_TASK_RESTRICT;
        e = launch_transfer(r, g->dev, c->dev, r ? t0.ch[0] : t0.ch[1], r ? t0.ch[1] : t0.ch[0], t0.param[0],
                            nd.check_activation ? 1 : 0, E().verify_demoted && !nd.check_activation ? 1 : 0, s);
        break;
    }
    case AT_TASK_ADVECT:
    case AT_TASK_P2G:
    case AT_TASK_G2P:
    case AT_TASK_P2G_MLS:
    case AT_TASK_G2P_APIC: {
        bool mpm = false;
        for (const Member &m : nd.members) {
            const int k = tasks[m.task].kind;
            mpm |= k == AT_TASK_P2G_MLS || k == AT_TASK_G2P_APIC;
        }
        if (mpm) {
            MpmProg mp{};
            mp.act_mode = nd.act_mode;
            mp.np = t0.n;
            mp.keep = 3u;
            for (const Member &m : nd.members) {
                const at_task &t = tasks[m.task];
                mp.x = (float *)t.ext[0];
                mp.v = (float *)t.ext[1];
                if (t.kind == AT_TASK_G2P_APIC) {
                    mp.steps |= PS_G2P;
                    mp.C = (float *)t.ext[2];
                    mp.keep = m.keep & 3u;
                    mp.gsrc = task_grid(t)->dev;
                    mp.inv_dx_src = (float)(1.0 / (double)t.param[0]);
                    mp.ch_vsrc = t.ch[0];
                } else if (t.kind == AT_TASK_ADVECT) {
                    mp.steps |= PS_ADVECT;
                    mp.adv_dt = t.param[0];
                } else {
                    mp.steps |= PS_P2G;
                    mp.C = (float *)t.ext[2];
                    mp.F = (float *)t.ext[3];
                    mp.gdst = task_grid(t)->dev;
                    mp.inv_dx_dst = (float)(1.0 / (double)t.param[0]);
                    mp.dt = t.param[1];
                    mp.mass = t.param[2];
                    mp.vol = t.param[3];
                    mp.mu = t.param[4];
                    mp.lam = t.param[5];
                    mp.ch_m = t.ch[0];
                    mp.ch_mv = t.ch[1];
                }
            }
            if (mp.np == 0) return AT_OK;
            if (mp.steps & PS_ADVECT) E().pos_writes[mp.x] += 1;
            e = launch_mpm(mp, s);
            break;
        }
        PartProg pp{};
        pp.act_mode = nd.act_mode;
        pp.np = t0.n;
        for (const Member &m : nd.members) {
            const at_task &t = tasks[m.task];
            pp.x = (float *)t.ext[0];
            if (t.kind == AT_TASK_G2P) {
                pp.steps |= PS_G2P;
                pp.v = (float *)t.ext[1];
                pp.gsrc = task_grid(t)->dev;
                pp.inv_dx_src = (float)(1.0 / (double)t.param[0]);
                pp.ch_vsrc = t.ch[0];
            } else if (t.kind == AT_TASK_ADVECT) {
                pp.steps |= PS_ADVECT;
                pp.v = (float *)t.ext[1];
                pp.dt = t.param[0];
            } else {
                pp.steps |= PS_P2G;
                pp.v = (float *)t.ext[1];
                pp.m = (const float *)t.ext[2];
                pp.gdst = task_grid(t)->dev;
                pp.inv_dx_dst = (float)(1.0 / (double)t.param[0]);
                pp.ch_m = t.ch[0];
                pp.ch_mv = t.ch[1];
            }
        }
        if (pp.np == 0) return AT_OK;
        at_grid_s *src = nullptr, *dst = nullptr;
        for (const Member &m : nd.members) {
            const at_task &t = tasks[m.task];
            if (t.kind == AT_TASK_G2P) src = const_cast<at_grid_s *>(task_grid(t));
            if (t.kind == AT_TASK_P2G) dst = const_cast<at_grid_s *>(task_grid(t));
        }
        Engine &en = E();
        int ndisp = 1;
        if (en.static_ws && dst) {
            // bins in the library's static array instead of the grid's workspace
            GridDev wsd = dst->dev;
            e = static_bin_workspace(wsd, pp.np, s);
            if (e != hipSuccess) return hip_fail(e, "static binning workspace");
            E().dispatches.fetch_add(1);
            pp.gdst = wsd;
            pp.gbin_s = wsd;
            e = launch_particles(pp, s, &ndisp);
            if (e != hipSuccess) return hip_fail(e, "kernel launch");
            // the grid's own workspace no longer holds its latest bins
            dst->bins_np = 0;
            dst->ws_gen += 1;
            E().dispatches.fetch_add(ndisp);
            return AT_OK;
        }
        const bool bin_dst = dst && dst->dev.pcap >= pp.np;
        // The gather may go through the bins of the source grid's last
        // binned scatter when it had exactly these many particles (the bins
        // then hold each index once) and the workspace holding them has not
        // been rebinned or cleared since.
        at_grid_s *own = src && src->bins_np == pp.np ? live_grid(src->bins_owner) : nullptr;
        if (own && (own->ws_gen != src->bins_owner_gen || own->dev.R != src->dev.R)) own = nullptr;
        // (a scatter of the same node that bins into that workspace runs in
        // later dispatches, after the gather has read it)
        pp.g2p_bins = own && en.g2p_bins ? 1 : 0;
        // the records' positions are current when they were written in this
        // window from this array and nothing has advected it since
        const auto pw = en.pos_writes.find(pp.x);
        const int64_t writes = pw == en.pos_writes.end() ? 0 : pw->second;
        pp.g2p_rec_x = pp.g2p_bins && src->bins_window == en.window_seq && src->bins_x == pp.x &&
                       src->bins_writes == writes ? 1 : 0;
        if (pp.g2p_bins) pp.gbin_g = own->dev;
        // A gather-advect-scatter node whose gather goes through current
        // records may scatter over the same bins (the gather updates the
        // records first), up to bin_reuse times before the particles are
        // binned again.
        pp.p2g_reuse = bin_dst && pp.g2p_rec_x && dst != src && own->bins_age < en.bin_reuse &&
                       own->dev.R == dst->dev.R && own->bins_inv_dx == pp.inv_dx_dst ? 1 : 0;
        pp.gbin_s = pp.p2g_reuse ? own->dev : (dst ? dst->dev : GridDev{});
        e = launch_particles(pp, s, &ndisp);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        const int64_t after = writes + ((pp.steps & PS_ADVECT) ? 1 : 0);
        if (pp.steps & PS_ADVECT) en.pos_writes[pp.x] = after;
        if (bin_dst) {
            dst->bins_np = pp.np;
            dst->bins_x = pp.x;
            dst->bins_window = en.window_seq;
            dst->bins_writes = after;
            if (pp.p2g_reuse) {
                own->bins_age += 1;
                dst->bins_owner = own->uid;
                dst->bins_owner_gen = own->ws_gen;
            } else {
                dst->ws_gen += 1;
                dst->bins_age = 0;
                dst->bins_inv_dx = pp.inv_dx_dst;
                dst->bins_owner = dst->uid;
                dst->bins_owner_gen = dst->ws_gen;
            }
        }
        E().dispatches.fetch_add(ndisp);
        return AT_OK;
    }
    default:
        return fail(AT_E_INVALID, "cannot execute task kind %d", t0.kind);
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    E().dispatches.fetch_add(1);
    return AT_OK;
}

void fill_stats(at_stats *st, int ntasks, const std::vector<Node> &nodes, const PlanCounters &c, int64_t disp,
                double us, int64_t hits) {
    if (!st) return;
    st->tasks_in = ntasks;
    st->tasks_launched = (int64_t)nodes.size();
    st->dispatches = disp;
    st->listgens_removed = c.listgens_removed;
    st->activations_demoted = c.activations_demoted;
    st->fusions = c.fusions;
    st->stores_eliminated = c.stores_eliminated;
    st->plan_cache_hits = hits;
    st->optimizer_us = us;
}

// Plan a window (no side effects on the engine unless `commit`).
at_status plan_window(const at_task *tasks, int ntasks, uint32_t flags, std::vector<Node> &nodes, PlanCounters &ctr,
                      int64_t &hits) {
    Engine &en = E();
    for (int i = 0; i < ntasks; ++i) {
        const std::string msg = validate_task(tasks[i]);
        if (!msg.empty()) return fail(AT_E_INVALID, "task %d: %s", i, msg.c_str());
    }
    hits = 0;
    Planner P(tasks, ntasks, flags, en.max_fuse, en.fuse_batch);
    if (flags == 0) {
        P.build_eager();
        nodes = std::move(P.nodes);
        ctr = PlanCounters{};
        return AT_OK;
    }
    const uint64_t key = hash_window(tasks, ntasks, flags, en.max_fuse);
    std::vector<uint8_t> fp = Planner::fingerprint(tasks, ntasks, en.persist);
    if (en.plan_cache) {
        auto it = en.cache.find(key);
        if (it != en.cache.end() && it->second.fp == fp) {
            nodes = it->second.nodes;
            ctr = it->second.counters;
            hits = 1;
            return AT_OK;
        }
    }
    P.build_eager();
    P.optimize(en.persist);
    nodes = std::move(P.nodes);
    ctr = P.counters;
    if (en.plan_cache) {
        if (en.cache.size() > 4096) en.cache.clear();
        en.cache[key] = CacheEntry{std::move(fp), nodes, ctr};
    }
    return AT_OK;
}

hipEvent_t take_event() {
    Engine &en = E();
    if (!en.ev_free.empty()) {
        hipEvent_t e = en.ev_free.back();
        en.ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

bool node_on_device(const Node &nd, const at_task *tasks) {
    for (const Member &m : nd.members) {
        const at_grid_s *g = task_grid(tasks[m.task]);
        if (g && g->virt) return false;
    }
    return true;
}

// Windows whose plan came from the plan cache and whose launches depend on
// nothing but the tasks and the plan -- struct-fors and two-level transfers
// (no list generation, whose launch carries a per-launch epoch; no
// activation; no particle task, whose binning state the host decides per
// launch) -- are captured once into a HIP graph on a side stream and
// replayed on the caller's stream afterwards: one host call instead of one
// per launch.  Windows of fewer than kGraphMinLaunches launches run directly:
// measured on the 20-step diffusion windows, a graph launch of a handful of
// kernels costs the host more than launching them.  The key covers the
// window, its plan, the neighbour-table choice of every node and the
// kernel-selection options.
constexpr size_t kGraphMinLaunches = 16;   // below this, direct launches cost the host less than a graph launch

bool graph_eligible(const std::vector<Node> &nodes, const at_task *tasks) {
    if (nodes.size() < kGraphMinLaunches) return false;
    for (const Node &nd : nodes)
        for (const Member &m : nd.members) {
            const int k = tasks[m.task].kind;
            if (k != AT_TASK_STENCIL && k != AT_TASK_RESTRICT && k != AT_TASK_PROLONG) return false;
        }
    return true;
}

uint64_t graph_key(const at_task *tasks, int ntasks, uint32_t flags, const std::vector<Node> &nodes,
                   const std::vector<uint8_t> &tables) {
    auto mixk = [](uint64_t h, uint64_t v) {
        h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
        return h * 0xff51afd7ed558ccdull;
    };
    uint64_t h = hash_window(tasks, ntasks, flags, E().max_fuse);
    for (size_t i = 0; i < nodes.size(); ++i) {
        const Node &nd = nodes[i];
        h = mixk(h, 0x4e0d3ull ^ nd.members.size());
        for (const Member &m : nd.members) h = mixk(mixk(h, (uint64_t)m.task), m.keep);
        h = mixk(h, (uint64_t)nd.check_activation | ((uint64_t)(uint32_t)nd.act_mode << 8) |
                        ((uint64_t)tables[i] << 40));
    }
    h = mixk(h, (uint64_t)(uint32_t)struct_for_kernel());
    return mixk(h, (uint64_t)(uint32_t)struct_for_grid_size_override());
}

void drop_graphs(bool sync) {
    Engine &en = E();
    if (en.graph_cache.empty()) return;
    if (sync) (void)hipDeviceSynchronize();
    for (auto &kv : en.graph_cache) (void)hipGraphExecDestroy(kv.second.exec);
    en.graph_cache.clear();
}

// Replays (or captures, then launches) the window's graph; false when the
// window is not eligible or capture failed (the caller then launches
// directly, nothing having run).
bool run_as_graph(const std::vector<Node> &nodes, const at_task *tasks, int ntasks, uint32_t flags,
                  const std::vector<uint8_t> &tables, hipStream_t s, at_status &st) {
    Engine &en = E();
    st = AT_OK;
    if (!en.graphs || en.timing || !graph_eligible(nodes, tasks)) return false;
    const uint64_t key = graph_key(tasks, ntasks, flags, nodes, tables);
    auto it = en.graph_cache.find(key);
    if (it == en.graph_cache.end()) {
        if (!en.capture_stream && hipStreamCreateWithFlags(&en.capture_stream, hipStreamNonBlocking) != hipSuccess) {
            en.capture_stream = nullptr;
            return false;
        }
        if (en.graph_cache.size() >= 64) drop_graphs(true);
        hipStream_t cs = en.capture_stream;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
        const int64_t d0 = en.dispatches.load();
        at_status est = AT_OK;
        for (size_t i = 0; i < nodes.size() && est == AT_OK; ++i) est = execute_node(nodes[i], tasks, tables[i] != 0, cs);
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        const int64_t nd = en.dispatches.load() - d0;
        en.dispatches.fetch_sub(nd);   // counted when the graph runs
        hipGraphExec_t exec = nullptr;
        const bool ok = est == AT_OK && ee == hipSuccess && graph &&
                        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        if (!ok) {
            (void)hipGetLastError();
            return false;
        }
        Engine::Graph G{exec, nd, {}};
        for (int i = 0; i < ntasks; ++i)
            for (const at_grid_s *g : {(const at_grid_s *)tasks[i].grid, (const at_grid_s *)tasks[i].grid2})
                if (g && std::find(G.uids.begin(), G.uids.end(), g->uid) == G.uids.end()) G.uids.push_back(g->uid);
        it = en.graph_cache.emplace(key, std::move(G)).first;
    }
    const hipError_t e = hipGraphLaunch(it->second.exec, s);
    if (e != hipSuccess) {
        st = hip_fail(e, "graph launch");
        return true;
    }
    en.dispatches.fetch_add(it->second.dispatches);
    return true;
}

// Checks a window shares between the synchronous and the asynchronous
// path; any_virt: it holds planning handles (it then launches nothing).
at_status check_window(const at_task *tasks, int ntasks, uint32_t flags, bool &any_virt) {
    if (ntasks < 0 || (ntasks > 0 && !tasks)) return fail(AT_E_INVALID, "bad task array");
    if (flags & ~AT_OPT_ALL) return fail(AT_E_INVALID, "unknown optimizer flags");
    // a window on planning handles only records engine state; its tasks
    // without a grid (advection) must not launch on their placeholder arrays
    bool any_dev = false;
    any_virt = false;
    for (int i = 0; i < ntasks; ++i)
        for (const at_grid_s *g : {(const at_grid_s *)tasks[i].grid, (const at_grid_s *)tasks[i].grid2})
            if (g) (g->virt ? any_virt : any_dev) = true;
    if (any_virt && any_dev) return fail(AT_E_INVALID, "a window mixes planning handles and device grids");
    return AT_OK;
}

// The launch half of a window: its planned nodes in order on stream s.
at_status launch_window(const std::vector<Node> &nodes, const at_task *tasks, int ntasks, uint32_t flags,
                        const std::vector<uint8_t> &tables, int64_t hits, bool any_virt, hipStream_t s) {
    Engine &en = E();
    ++en.window_seq;
    en.pos_writes.clear();
    at_status st = AT_OK;
    if (!any_virt && hits > 0 && run_as_graph(nodes, tasks, ntasks, flags, tables, s, st)) return st;
    for (size_t i = 0; i < nodes.size() && !any_virt; ++i) {
        const Node &nd = nodes[i];
        hipEvent_t ea = nullptr;
        if (en.timing && node_on_device(nd, tasks)) {
            ea = take_event();
            if (ea && hipEventRecord(ea, s) != hipSuccess) ea = nullptr;
        }
        st = execute_node(nd, tasks, tables[i] != 0, s);
        if (ea) {
            hipEvent_t eb = take_event();
            if (eb && hipEventRecord(eb, s) == hipSuccess) {
                const at_task &t0 = tasks[nd.members[0].task];
                en.timed.push_back({t0.kind, t0.op, (int32_t)nd.members.size(), ea, eb});
            } else {
                en.ev_free.push_back(ea);
                if (eb) en.ev_free.push_back(eb);
            }
        }
        if (st != AT_OK) return st;
    }
    return AT_OK;
}

at_status run_window(const at_task *tasks, int ntasks, uint32_t flags, at_stats *stats, hipStream_t s) {
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    bool any_virt = false;
    at_status st = check_window(tasks, ntasks, flags, any_virt);
    if (st != AT_OK) return st;
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<Node> nodes;
    PlanCounters ctr;
    int64_t hits = 0;
    st = plan_window(tasks, ntasks, flags, nodes, ctr, hits);
    if (st != AT_OK) return st;
    const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    const int64_t d0 = en.dispatches.load();
    const std::vector<uint8_t> tables = neighbour_tables_valid(nodes, tasks, en.persist);
    st = launch_window(nodes, tasks, ntasks, flags, tables, hits, any_virt, s);
    Planner::commit(nodes, tasks, en.persist);
    if (st != AT_OK) return st;
    fill_stats(stats, ntasks, nodes, ctr, en.dispatches.load() - d0, us, hits);
    return AT_OK;
}

// ------------------------------------------------- asynchronous pipeline
// Flushed windows are planned by an optimizer thread, in flush order, and
// launched by a launcher thread, so the optimizer plans a window while the
// previous one is being launched and the caller goes on enqueueing (the
// paper's asynchronous engine, Section 7).  Planning touches only the
// persistent graph state and the plan cache; launching only the per-launch
// state (bin reuse, graphs, timing).  Every other engine call first waits
// for the pipeline to empty, so program order holds on every stream.

void add_stats(at_stats &a, const at_stats &b) {
    a.tasks_in += b.tasks_in;
    a.tasks_launched += b.tasks_launched;
    a.dispatches += b.dispatches;
    a.listgens_removed += b.listgens_removed;
    a.activations_demoted += b.activations_demoted;
    a.fusions += b.fusions;
    a.stores_eliminated += b.stores_eliminated;
    a.plan_cache_hits += b.plan_cache_hits;
    a.optimizer_us += b.optimizer_us;
}

void optimizer_loop(AsyncPipe *p) {
    Engine &en = E();
    for (;;) {
        std::unique_ptr<PendingWindow> w;
        bool failed;
        {
            std::unique_lock<std::mutex> lk(p->mu);
            p->cv.wait(lk, [&] { return !p->to_plan.empty(); });
            w = std::move(p->to_plan.front());
            p->to_plan.pop_front();
            ++p->busy;
            failed = p->err != AT_OK;
        }
        at_status st = AT_OK;
        if (!failed) {   // after a failure, windows are dropped until it is reported
            const auto t0 = std::chrono::steady_clock::now();
            st = plan_window(w->tasks.data(), (int)w->tasks.size(), w->flags, w->nodes, w->ctr, w->hits);
            if (st == AT_OK) {
                w->tables = neighbour_tables_valid(w->nodes, w->tasks.data(), en.persist);
                Planner::commit(w->nodes, w->tasks.data(), en.persist);
            }
            w->us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
        }
        std::lock_guard<std::mutex> lk(p->mu);
        --p->busy;
        if (st != AT_OK && p->err == AT_OK) {
            p->err = st;
            p->msg = at_last_error();
        }
        if (st == AT_OK && !failed) p->to_launch.push_back(std::move(w));
        p->cv.notify_all();
    }
}

void launcher_loop(AsyncPipe *p) {
    Engine &en = E();
    int device = -1;
    for (;;) {
        std::unique_ptr<PendingWindow> w;
        bool failed;
        {
            std::unique_lock<std::mutex> lk(p->mu);
            p->cv.wait(lk, [&] { return !p->to_launch.empty(); });
            w = std::move(p->to_launch.front());
            p->to_launch.pop_front();
            ++p->busy;
            failed = p->err != AT_OK;
        }
        at_status st = AT_OK;
        at_stats one{};
        if (!failed) {
            if (w->device >= 0 && w->device != device) {
                const hipError_t e = hipSetDevice(w->device);
                if (e != hipSuccess) st = hip_fail(e, "launcher thread device");
                else device = w->device;
            }
            if (st == AT_OK) {
                const int64_t d0 = en.dispatches.load();
                st = launch_window(w->nodes, w->tasks.data(), (int)w->tasks.size(), w->flags, w->tables, w->hits,
                                   w->any_virt, w->stream);
                fill_stats(&one, (int)w->tasks.size(), w->nodes, w->ctr, en.dispatches.load() - d0, w->us, w->hits);
            }
        }
        std::lock_guard<std::mutex> lk(p->mu);
        --p->busy;
        if (st != AT_OK && p->err == AT_OK) {
            p->err = st;
            p->msg = at_last_error();
        }
        if (st == AT_OK && !failed) add_stats(p->sum, one);
        p->cv.notify_all();
    }
}

void start_pipe() {
    Engine &en = E();
    if (en.pipe) return;
    en.pipe.reset(new AsyncPipe());
    AsyncPipe *p = en.pipe.get();
    p->optimizer = std::thread(optimizer_loop, p);
    p->launcher = std::thread(launcher_loop, p);
    p->optimizer.detach();
    p->launcher.detach();
}

// Waits until every submitted window has been launched.  Returns (and
// clears) the first failure of a window since the last report when
// `report`; otherwise it stays for a later report.
at_status drain_pipe(bool report) {
    Engine &en = E();
    AsyncPipe *p = en.pipe.get();
    if (!p) return AT_OK;
    std::unique_lock<std::mutex> lk(p->mu);
    p->cv.wait(lk, [&] { return p->to_plan.empty() && p->to_launch.empty() && p->busy == 0; });
    if (!report || p->err == AT_OK) return AT_OK;
    const at_status e = p->err;
    const std::string msg = p->msg;
    p->err = AT_OK;
    p->msg.clear();
    return fail(e, "%s", msg.c_str());
}

// Hands a window to the pipeline (the caller holds en.mu).  A failure of an
// earlier window is reported here first, and this window is then dropped.
at_status submit_window(const at_task *tasks, int ntasks, uint32_t flags, at_stats *stats, hipStream_t s) {
    Engine &en = E();
    if (stats) std::memset(stats, 0, sizeof *stats);
    bool any_virt = false;
    at_status st = check_window(tasks, ntasks, flags, any_virt);
    if (st != AT_OK) return st;
    for (int i = 0; i < ntasks; ++i) {
        const std::string msg = validate_task(tasks[i]);
        if (!msg.empty()) return fail(AT_E_INVALID, "task %d: %s", i, msg.c_str());
    }
    start_pipe();
    AsyncPipe *p = en.pipe.get();
    auto w = std::unique_ptr<PendingWindow>(new PendingWindow());
    w->tasks.assign(tasks, tasks + ntasks);
    w->flags = flags;
    w->stream = s;
    w->any_virt = any_virt;
    int dev = -1;
    if (!any_virt && hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        dev = -1;
    }
    w->device = dev;
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->err != AT_OK) {
        const at_status e = p->err;
        const std::string msg = p->msg;
        p->err = AT_OK;
        p->msg.clear();
        return fail(e, "an earlier asynchronous window failed: %s", msg.c_str());
    }
    if (stats) stats->tasks_in = ntasks;
    p->to_plan.push_back(std::move(w));
    p->cv.notify_all();
    return AT_OK;
}

// A window from the queue or a caller: through the pipeline when
// asynchronous, else planned and launched here.
at_status dispatch_window(const at_task *tasks, int ntasks, uint32_t flags, at_stats *stats, hipStream_t s) {
    if (E().async) return submit_window(tasks, ntasks, flags, stats, s);
    return run_window(tasks, ntasks, flags, stats, s);
}

at_status run_one(const at_task &t, hipStream_t s) {
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    if (!en.queue.empty()) {
        // keep program order with queued work
        at_status st = dispatch_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, nullptr, en.queue_stream);
        en.queue.clear();
        if (st != AT_OK) return st;
    }
    at_status st = drain_pipe(true);
    if (st != AT_OK) return st;
    return run_window(&t, 1, 0, nullptr, s);
}

at_task blank_task(int kind, at_grid g) {
    at_task t;
    std::memset(&t, 0, sizeof t);
    t.kind = kind;
    t.grid = g;
    for (int q = 0; q < 8; ++q) t.ch[q] = -1;
    return t;
}

// Bump the versions of states written outside tasks (setup copies, clears).
void bump(uint64_t uid, uint8_t kind, int32_t ch) {
    E().persist.version[StateKey{uid, ch, kind}] += 1;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

at_status at_grid_footprint(const at_grid_desc *desc, size_t *bytes) {
    if (!bytes) return fail(AT_E_INVALID, "null output");
    Layout L;
    at_status st = layout_of(desc, L);
    if (st != AT_OK) return st;
    *bytes = L.total;
    return AT_OK;
}

at_status at_grid_create(const at_grid_desc *desc, void *dev_buf, size_t bytes, hipStream_t stream, at_grid *out) {
    if (!out) return fail(AT_E_INVALID, "null output handle");
    *out = nullptr;
    Layout L;
    at_status st = layout_of(desc, L);
    if (st != AT_OK) return st;
    const bool virt = dev_buf == nullptr;
    if (!virt) {
        if (bytes < L.total) return fail(AT_E_INVALID, "buffer of %zu bytes below the footprint %zu", bytes, L.total);
        if (((uintptr_t)dev_buf & 255) != 0) return fail(AT_E_INVALID, "grid buffer must be 256-byte aligned");
    }
    at_grid g = new at_grid_s();
    g->desc = *desc;
    g->virt = virt;
    g->bytes = L.total;
    g->list_cap = L.list_cap;
    g->listgen_epoch = 0;
    GridDev &d = g->dev;
    d.R = L.R;
    d.R2 = L.R * L.R;
    d.kind = desc->root_kind;
    d.cap = L.cap;
    d.ncells = L.ncells;
    d.ch_stride = (int64_t)L.cap * kBV;
    if (!virt) {
        char *b = (char *)dev_buf;
        d.hdr = (int32_t *)(b + L.hdr);
        d.scan = (uint64_t *)(b + L.scan);
        d.bits = (uint32_t *)(b + L.bits);
        d.ptr = desc->root_kind == AT_ROOT_POINTER ? (int32_t *)(b + L.ptr) : nullptr;
        d.list = (int32_t *)(b + L.list);
        d.pcap = L.pcap;
        d.pcount = L.pcap ? (int32_t *)(b + L.pcount) : nullptr;
        d.poff = L.pcap ? (int32_t *)(b + L.poff) : nullptr;
        d.pbins = L.pcap ? (int4 *)(b + L.pbins) : nullptr;
        d.pkr = L.pcap ? (int2 *)(b + L.pkr) : nullptr;
        d.pstage = L.pcap ? (float4 *)(b + L.pstage) : nullptr;
        d.pout = L.pcap ? (int32_t *)(b + L.pout) : nullptr;
        d.chan = (float *)(b + L.chan);
        hipError_t e = hipMemsetAsync(dev_buf, 0, L.total, stream);
        if (e == hipSuccess && d.ptr) e = hipMemsetAsync(d.ptr, 0xff, (size_t)L.ncells * 4, stream);
        if (e != hipSuccess) {
            delete g;
            return hip_fail(e, "grid initialisation");
        }
        E().dispatches.fetch_add(d.ptr ? 2 : 1);
    }
    {
        std::lock_guard<std::recursive_mutex> lk(E().mu);
        drain_pipe(false);   // the launcher reads the live-grid map
        g->uid = E().next_uid++;
        E().live[g->uid] = g;
    }
    *out = g;
    return AT_OK;
}

at_status at_grid_destroy(at_grid grid) {
    if (!grid) return fail(AT_E_INVALID, "null grid handle");
    {
        Engine &en = E();
        std::lock_guard<std::recursive_mutex> lk(en.mu);
        drain_pipe(false);
        for (const at_task &t : en.queue)
            if (t.grid == grid || t.grid2 == grid) return fail(AT_E_STATE, "grid has queued tasks; flush first");
        en.persist.forget_grid(grid->uid);
        en.live.erase(grid->uid);
        for (auto it = en.graph_cache.begin(); it != en.graph_cache.end();) {
            const auto &u = it->second.uids;
            if (std::find(u.begin(), u.end(), grid->uid) != u.end()) {
                (void)hipGraphExecDestroy(it->second.exec);   // freed once any launch in flight completes
                it = en.graph_cache.erase(it);
            } else {
                ++it;
            }
        }
    }
    delete grid;
    return AT_OK;
}

at_status at_grid_views(at_grid grid, float **ch_base, const int32_t **list, const int32_t **count, const void **root) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    if (ch_base)
        for (int c = 0; c < grid->desc.channels; ++c) ch_base[c] = grid->dev.chan + (int64_t)c * grid->dev.ch_stride;
    if (list) *list = grid->dev.list;
    if (count) *count = grid->dev.hdr + HDR_COUNT;
    if (root) *root = grid->desc.root_kind == AT_ROOT_POINTER ? (const void *)grid->dev.ptr : (const void *)grid->dev.bits;
    return AT_OK;
}

at_status at_grid_get_info(at_grid grid, at_grid_info *info) {
    at_status st = check_grid(grid, false);
    if (st != AT_OK) return st;
    if (!info) return fail(AT_E_INVALID, "null output");
    info->n = grid->desc.n[0];
    info->R = grid->dev.R;
    info->root_kind = grid->desc.root_kind;
    info->channels = grid->desc.channels;
    info->capacity_blocks = grid->dev.cap;
    info->list_capacity = grid->list_cap;
    info->ncells = grid->dev.ncells;
    info->bytes = grid->bytes;
    return AT_OK;
}

at_status at_grid_clear(at_grid grid, hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    if (!en.queue.empty()) {
        st = run_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, nullptr, en.queue_stream);
        en.queue.clear();
        if (st != AT_OK) return st;
    }
    const GridDev &d = grid->dev;
    hipError_t e = hipMemsetAsync(d.hdr, 0, 2 * sizeof(int32_t), stream);   // count and bump
    if (e == hipSuccess) e = hipMemsetAsync(d.bits, 0, ((d.ncells + 31) / 32) * 4, stream);
    if (e == hipSuccess && d.ptr) e = hipMemsetAsync(d.ptr, 0xff, (size_t)d.ncells * 4, stream);
    if (e == hipSuccess) e = hipMemsetAsync(d.chan, 0, (size_t)grid->desc.channels * d.ch_stride * sizeof(float), stream);
    if (e == hipSuccess && d.pcount) e = hipMemsetAsync(d.pcount, 0, (size_t)d.ncells * sizeof(int32_t), stream);
    if (e == hipSuccess && d.pcount) e = hipMemsetAsync(d.hdr + HDR_NBINS, 0, 4 * sizeof(int32_t), stream);
    if (e != hipSuccess) return hip_fail(e, "grid clear");
    en.dispatches.fetch_add((d.ptr ? 4 : 3) + (d.pcount ? 2 : 0));
    grid->bins_np = 0;
    grid->ws_gen += 1;
    en.persist.deactivate_grid(grid->uid);
    for (int c = 0; c < grid->desc.channels; ++c) bump(grid->uid, ST_VALUE, c);
    bump(grid->uid, ST_ALLOC, -1);
    return AT_OK;
}

at_status at_device_status(at_grid grid, hipStream_t stream, int32_t clear, int32_t *bits) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    {
        std::lock_guard<std::recursive_mutex> lk(E().mu);
        drain_pipe(false);
    }
    if (!bits) return fail(AT_E_INVALID, "null output");
    hipError_t e = hipMemcpyAsync(bits, grid->dev.hdr + HDR_ERR, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess && clear) {
        e = hipMemsetAsync(grid->dev.hdr + HDR_ERR, 0, sizeof(int32_t), stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    if (e != hipSuccess) return hip_fail(e, "device status");
    return AT_OK;
}

at_status at_active_count(at_grid grid, hipStream_t stream, int64_t *count) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    {
        std::lock_guard<std::recursive_mutex> lk(E().mu);
        drain_pipe(false);
    }
    if (!count) return fail(AT_E_INVALID, "null output");
    hipError_t e = launch_popcount(grid->dev, stream);
    int32_t v = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&v, grid->dev.hdr + HDR_SCRATCH, sizeof v, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "active count");
    E().dispatches.fetch_add(1);
    *count = v;
    return AT_OK;
}

at_status at_activate(at_grid grid, const int32_t *d_ijk, int64_t n, int32_t coord_kind, hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    at_task t = blank_task(AT_TASK_ACTIVATE, grid);
    t.op = coord_kind;
    t.ext[0] = (void *)d_ijk;
    t.n = n;
    return run_one(t, stream);
}

at_status at_listgen(at_grid grid, hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    return run_one(blank_task(AT_TASK_LISTGEN, grid), stream);
}

at_status at_run_stencil(at_grid grid, int32_t op, const int32_t *ch, const float *params, int32_t check_activation,
                         hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    if (!ch) return fail(AT_E_INVALID, "null channel array");
    at_task t = blank_task(AT_TASK_STENCIL, grid);
    t.op = op;
    if (op == AT_OP_FILL) {
        for (int q = 0; q < 8; ++q) {
            t.ch[q] = ch[q];
            if (ch[q] < 0) break;
        }
    } else {
        const int nc = op == AT_OP_LAP_UPDATE || op == AT_OP_AXPY || op == AT_OP_COPY ? 2
                     : op == AT_OP_INC ? 1 : op == AT_OP_DIFFUSE_ADJ || op == AT_OP_MACCORMACK ? 5 : 3;
        if (op < AT_OP_LAP_UPDATE || op > AT_OP_MPM_GRID) return fail(AT_E_INVALID, "unknown op %d", op);
        for (int q = 0; q < nc; ++q) t.ch[q] = ch[q];
    }
    if (params) {
        const int np = op == AT_OP_ADVECT || op == AT_OP_MACCORMACK ? 2 : op == AT_OP_MPM_GRID ? 3 : 1;
        for (int q = 0; q < np; ++q) t.param[q] = params[q];
    }
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    if (check_activation) return run_one(t, stream);
    // demoted form requested explicitly: plan with activation demotion only
    if (!en.queue.empty()) {
        st = run_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, nullptr, en.queue_stream);
        en.queue.clear();
        if (st != AT_OK) return st;
    }
    return run_window(&t, 1, AT_OPT_AD, nullptr, stream);
}

at_status at_advect(float *d_x, const float *d_v, int64_t np, float dt, hipStream_t stream) {
    at_task t = blank_task(AT_TASK_ADVECT, nullptr);
    t.ext[0] = d_x;
    t.ext[1] = (void *)d_v;
    t.n = np;
    t.param[0] = dt;
    t.flags = AT_TASKF_LOOP_UNIQUE;
    return run_one(t, stream);
}

at_status at_p2g(at_grid grid, const float *d_x, const float *d_v, const float *d_m, int64_t np, float dx,
                 const int32_t *ch, int32_t activation, hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    if (!ch) return fail(AT_E_INVALID, "null channel array");
    at_task t = blank_task(AT_TASK_P2G, grid);
    t.op = activation;
    t.ext[0] = (void *)d_x;
    t.ext[1] = (void *)d_v;
    t.ext[2] = (void *)d_m;
    t.n = np;
    t.param[0] = dx;
    t.ch[0] = ch[0];
    t.ch[1] = ch[1];
    t.flags = AT_TASKF_LOOP_UNIQUE;
    return run_one(t, stream);
}

at_status at_p2g_static(at_grid grid, const float *d_x, const float *d_v, const float *d_m, int64_t np, float dx,
                        const int32_t *ch, int32_t activation, hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    if (!ch) return fail(AT_E_INVALID, "null channel array");
    if (np < 0) return fail(AT_E_INVALID, "negative particle count");
    if (np > AT_STATIC_MAX_PARTICLES)
        return fail(AT_E_INVALID, "%lld particles exceed the static workspace's limit of %d", (long long)np,
                    AT_STATIC_MAX_PARTICLES);
    if (grid->dev.ncells > AT_STATIC_MAX_CELLS)
        return fail(AT_E_INVALID, "%lld root cells exceed the static workspace's limit of %d",
                    (long long)grid->dev.ncells, AT_STATIC_MAX_CELLS);
    at_task t = blank_task(AT_TASK_P2G, grid);
    t.op = activation;
    t.ext[0] = (void *)d_x;
    t.ext[1] = (void *)d_v;
    t.ext[2] = (void *)d_m;
    t.n = np;
    t.param[0] = dx;
    t.ch[0] = ch[0];
    t.ch[1] = ch[1];
    t.flags = AT_TASKF_LOOP_UNIQUE;
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    if (!en.queue.empty()) {
        st = run_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, nullptr, en.queue_stream);
        en.queue.clear();
        if (st != AT_OK) return st;
    }
    en.static_ws = true;
    st = run_window(&t, 1, 0, nullptr, stream);
    en.static_ws = false;
    return st;
}

at_status at_p2g_mls(at_grid grid, const float *d_x, const float *d_v, const float *d_C, float *d_F, int64_t np,
                     float dx, float dt, float mass, float vol, float mu, float lambda, const int32_t *ch,
                     int32_t activation, hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    if (!ch) return fail(AT_E_INVALID, "null channel array");
    at_task t = blank_task(AT_TASK_P2G_MLS, grid);
    t.op = activation;
    t.ext[0] = (void *)d_x;
    t.ext[1] = (void *)d_v;
    t.ext[2] = (void *)d_C;
    t.ext[3] = d_F;
    t.n = np;
    const float prm[6] = {dx, dt, mass, vol, mu, lambda};
    for (int q = 0; q < 6; ++q) t.param[q] = prm[q];
    t.ch[0] = ch[0];
    t.ch[1] = ch[1];
    t.flags = AT_TASKF_LOOP_UNIQUE;
    return run_one(t, stream);
}

at_status at_g2p_apic(at_grid grid, const float *d_x, float *d_v, float *d_C, int64_t np, float dx, const int32_t *ch,
                      hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    if (!ch) return fail(AT_E_INVALID, "null channel array");
    at_task t = blank_task(AT_TASK_G2P_APIC, grid);
    t.ext[0] = (void *)d_x;
    t.ext[1] = d_v;
    t.ext[2] = d_C;
    t.n = np;
    t.param[0] = dx;
    t.ch[0] = ch[0];
    t.flags = AT_TASKF_LOOP_UNIQUE;
    return run_one(t, stream);
}

at_status at_g2p(at_grid grid, const float *d_x, float *d_v, int64_t np, float dx, const int32_t *ch,
                 hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    if (!ch) return fail(AT_E_INVALID, "null channel array");
    at_task t = blank_task(AT_TASK_G2P, grid);
    t.ext[0] = (void *)d_x;
    t.ext[1] = d_v;
    t.n = np;
    t.param[0] = dx;
    t.ch[0] = ch[0];
    t.flags = AT_TASKF_LOOP_UNIQUE;
    return run_one(t, stream);
}

at_status at_scatter_blocks(at_grid grid, int32_t ch, const int32_t *d_cells, const float *d_vals, int64_t n,
                            hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    if (ch < 0 || ch >= grid->desc.channels) return fail(AT_E_INVALID, "channel out of range");
    if (n < 0 || (n > 0 && (!d_cells || !d_vals))) return fail(AT_E_INVALID, "bad block arrays");
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    if (!en.queue.empty()) {
        st = run_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, nullptr, en.queue_stream);
        en.queue.clear();
        if (st != AT_OK) return st;
    }
    if (n == 0) return AT_OK;
    hipError_t e = launch_scatter_blocks(grid->dev, ch, d_cells, d_vals, n, stream);
    if (e != hipSuccess) return hip_fail(e, "scatter blocks");
    en.dispatches.fetch_add(1);
    bump(grid->uid, ST_MASK, -1);
    bump(grid->uid, ST_ALLOC, -1);
    bump(grid->uid, ST_VALUE, ch);
    return AT_OK;
}

at_status at_gather_blocks(at_grid grid, int32_t ch, const int32_t *d_cells, float *d_vals, int64_t n,
                           hipStream_t stream) {
    at_status st = check_grid(grid, true);
    if (st != AT_OK) return st;
    if (ch < 0 || ch >= grid->desc.channels) return fail(AT_E_INVALID, "channel out of range");
    if (n < 0 || (n > 0 && (!d_cells || !d_vals))) return fail(AT_E_INVALID, "bad block arrays");
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    if (!en.queue.empty()) {
        st = run_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, nullptr, en.queue_stream);
        en.queue.clear();
        if (st != AT_OK) return st;
    }
    if (n == 0) return AT_OK;
    hipError_t e = launch_gather_blocks(grid->dev, ch, d_cells, d_vals, n, stream);
    if (e != hipSuccess) return hip_fail(e, "gather blocks");
    en.dispatches.fetch_add(1);
    return AT_OK;
}

at_status at_run_sequence(const at_task *tasks, int32_t ntasks, uint32_t opt_flags, at_stats *stats,
                          hipStream_t stream) {
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    if (!en.queue.empty()) {
        at_status st = dispatch_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, nullptr, en.queue_stream);
        en.queue.clear();
        if (st != AT_OK) return st;
    }
    return dispatch_window(tasks, ntasks, opt_flags, stats, stream);
}

at_status at_variant_prepare(const at_task *tasks, int32_t ntasks, char *src, size_t cap, size_t *len) {
    if (ntasks < 2 || ntasks > kMaxOps || !tasks) return fail(AT_E_INVALID, "a variant takes 2 .. %d tasks", kMaxOps);
    if (cap > 0 && !src) return fail(AT_E_INVALID, "null source buffer");
    MicroProg prog{};
    prog.nops = ntasks;
    for (int32_t i = 0; i < ntasks; ++i) {
        const at_task &t = tasks[i];
        const std::string msg = validate_task(t);
        if (!msg.empty()) return fail(AT_E_INVALID, "task %d: %s", i, msg.c_str());
        if (t.kind != AT_TASK_STENCIL || t.grid != tasks[0].grid)
            return fail(AT_E_UNSUPPORTED, "task %d: variants cover struct-for tasks of one grid", i);
        MicroOp &op = prog.ops[i];
        op.op = t.op;
        for (int c = 0; c < 7; ++c) op.ch[c] = t.ch[c];
        op.p = t.param[0];
        op.keep = ~0u;
        op.p1 = t.param[1];
        op.p2 = t.param[2];
    }
    TileProg tp;
    if (!variant_eligible(prog) && !tile_prog(prog, tp))
        return fail(AT_E_UNSUPPORTED, "variants cover copy, axpy, inc, fill and normalise chains that save memory "
                                      "traffic, and advection tile programs");
    const at_grid_s *g0 = reinterpret_cast<const at_grid_s *>(tasks[0].grid);
    std::string s;
    if (!variant_prepare(prog, g0->desc.root_kind, s)) return fail(AT_E_UNSUPPORTED, "the variant did not compile");
    if (len) *len = s.size();
    if (cap > 0) {
        const size_t n = s.size() < cap - 1 ? s.size() : cap - 1;
        std::memcpy(src, s.data(), n);
        src[n] = 0;
    }
    return AT_OK;
}

at_status at_engine_sync(at_stats *stats) {
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    if (stats) std::memset(stats, 0, sizeof *stats);
    at_status st = drain_pipe(true);
    if (en.pipe) {
        std::lock_guard<std::mutex> pl(en.pipe->mu);
        if (stats) *stats = en.pipe->sum;
        en.pipe->sum = at_stats{};
    }
    return st;
}

at_status at_plan_sequence(const at_task *tasks, int32_t ntasks, uint32_t opt_flags, at_plan_entry *out,
                           int32_t capacity, int32_t *nout, at_stats *stats) {
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    if (ntasks < 0 || (ntasks > 0 && !tasks)) return fail(AT_E_INVALID, "bad task array");
    if (opt_flags & ~AT_OPT_ALL) return fail(AT_E_INVALID, "unknown optimizer flags");
    if (!nout || capacity < 0 || (capacity > 0 && !out)) return fail(AT_E_INVALID, "bad output array");
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<Node> nodes;
    PlanCounters ctr;
    int64_t hits = 0;
    // planning must not populate the cache with a plan that was never run
    drain_pipe(false);
    const bool cache = en.plan_cache;
    en.plan_cache = false;
    at_status st = plan_window(tasks, ntasks, opt_flags, nodes, ctr, hits);
    en.plan_cache = cache;
    if (st != AT_OK) return st;
    const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    *nout = (int32_t)nodes.size();
    if ((int32_t)nodes.size() > capacity) return fail(AT_E_INVALID, "plan has %zu entries, capacity %d", nodes.size(), capacity);
    for (size_t i = 0; i < nodes.size(); ++i) {
        const Node &nd = nodes[i];
        at_plan_entry &e = out[i];
        std::memset(&e, 0, sizeof e);
        e.kind = tasks[nd.members[0].task].kind;
        e.nmembers = (int32_t)nd.members.size();
        static_assert(AT_PLAN_MAX_MEMBERS >= kMaxOps, "a plan entry holds every member of a fused launch");
        for (size_t m = 0; m < nd.members.size() && m < AT_PLAN_MAX_MEMBERS; ++m) {
            e.members[m] = nd.members[m].task;
            e.keep[m] = nd.members[m].keep;
            if (nd.members[m].keep != ~0u) e.dropped |= 1u << m;
        }
        e.check_activation = nd.check_activation ? 1 : 0;
        e.activation_mode = nd.act_mode;
    }
    fill_stats(stats, ntasks, nodes, ctr, (int64_t)nodes.size(), us, hits);
    return AT_OK;
}

at_status at_enqueue(const at_task *task, hipStream_t stream) {
    if (!task) return fail(AT_E_INVALID, "null task");
    const std::string msg = validate_task(*task);
    if (!msg.empty()) return fail(AT_E_INVALID, "%s", msg.c_str());
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    if (!en.queue.empty() && stream != en.queue_stream) {
        at_status st = dispatch_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, nullptr, en.queue_stream);
        en.queue.clear();
        if (st != AT_OK) return st;
    }
    en.queue.push_back(*task);
    en.queue_stream = stream;
    if (en.flush_period > 0 && (int64_t)en.queue.size() >= en.flush_period) {
        at_status st = dispatch_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, nullptr, en.queue_stream);
        en.queue.clear();
        return st;
    }
    return AT_OK;
}

at_status at_flush(at_stats *stats, hipStream_t stream) {
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    if (en.queue.empty()) {
        if (stats) std::memset(stats, 0, sizeof *stats);
        return AT_OK;
    }
    (void)stream;
    at_status st = dispatch_window(en.queue.data(), (int)en.queue.size(), en.opt_flags, stats, en.queue_stream);
    en.queue.clear();
    return st;
}

at_status at_set_option(int32_t option, int64_t value) {
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    switch (option) {
    case AT_OPTION_ASYNC:
        if (value != 0 && value != 1) return fail(AT_E_INVALID, "async must be 0 or 1");
        en.async = value != 0;
        return AT_OK;
    case AT_OPTION_VARIANTS:
        if (value < 0 || value > 2) return fail(AT_E_INVALID, "variants must be 0, 1 or 2");
        set_variant_mode((int)value);
        return AT_OK;
    case AT_OPTION_VARIANTS_LOADED: return fail(AT_E_INVALID, "the number of loaded variants is read-only");
    case AT_OPTION_VERIFY_DEMOTED:
        if (value != 0 && value != 1) return fail(AT_E_INVALID, "verify demoted must be 0 or 1");
        // a captured graph holds the kernels of the other setting
        if (en.verify_demoted != (value != 0)) drop_graphs(true);
        en.verify_demoted = value != 0;
        return AT_OK;
    case AT_OPTION_MAX_FUSE_PER_TASK:
        if (value < 1 || value > 64) return fail(AT_E_INVALID, "max_fuse_per_task must be in 1..64");
        en.max_fuse = (int)value;
        en.cache.clear();
        return AT_OK;
    case AT_OPTION_FLUSH_PERIOD:
        if (value < 0) return fail(AT_E_INVALID, "flush period must be >= 0");
        en.flush_period = value;
        return AT_OK;
    case AT_OPTION_OPT_FLAGS:
        if (value < 0 || (value & ~(int64_t)AT_OPT_ALL)) return fail(AT_E_INVALID, "unknown optimizer flags");
        en.opt_flags = (uint32_t)value;
        return AT_OK;
    case AT_OPTION_PLAN_CACHE:
        en.plan_cache = value != 0;
        if (!en.plan_cache) en.cache.clear();
        return AT_OK;
    case AT_OPTION_STRUCT_FOR_WORKGROUPS:
        if (value < 0 || value > (1 << 20)) return fail(AT_E_INVALID, "workgroup count out of range");
        set_struct_for_grid_size((int)value);
        return AT_OK;
    case AT_OPTION_STRUCT_FOR_KERNEL:
        if (value < 0 || value > 2) return fail(AT_E_INVALID, "struct-for kernel form must be 0, 1 or 2");
        set_struct_for_kernel((int)value);
        return AT_OK;
    case AT_OPTION_BATCH_WAVES:
        if (value != 1 && value != 2 && value != 4) return fail(AT_E_INVALID, "batch waves must be 1, 2 or 4");
        set_batch_waves((int)value);
        return AT_OK;
    case AT_OPTION_G2P_BINS:
        if (value != 0 && value != 1) return fail(AT_E_INVALID, "g2p bins must be 0 or 1");
        en.g2p_bins = value != 0;
        return AT_OK;
    case AT_OPTION_BIN_REUSE:
        if (value < 0 || value > 1024) return fail(AT_E_INVALID, "bin reuse must be in 0..1024");
        en.bin_reuse = (int32_t)value;
        return AT_OK;
    case AT_OPTION_FUSE_BATCH:
        if (value != 0 && value != 1) return fail(AT_E_INVALID, "fuse batch must be 0 or 1");
        en.fuse_batch = value != 0;
        en.cache.clear();
        return AT_OK;
    case AT_OPTION_GRAPHS_CACHED: return fail(AT_E_INVALID, "the number of cached graphs is read-only");
    case AT_OPTION_GRAPHS:
        if (value != 0 && value != 1) return fail(AT_E_INVALID, "graphs must be 0 or 1");
        en.graphs = value != 0;   // cached graphs stay until reset or their grids go
        return AT_OK;
    default:
        return fail(AT_E_INVALID, "unknown option %d", option);
    }
}

at_status at_get_option(int32_t option, int64_t *value) {
    if (!value) return fail(AT_E_INVALID, "null output");
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    switch (option) {
    case AT_OPTION_MAX_FUSE_PER_TASK: *value = en.max_fuse; return AT_OK;
    case AT_OPTION_FLUSH_PERIOD: *value = en.flush_period; return AT_OK;
    case AT_OPTION_OPT_FLAGS: *value = en.opt_flags; return AT_OK;
    case AT_OPTION_PLAN_CACHE: *value = en.plan_cache ? 1 : 0; return AT_OK;
    case AT_OPTION_STRUCT_FOR_WORKGROUPS: *value = struct_for_grid_size_override(); return AT_OK;
    case AT_OPTION_STRUCT_FOR_KERNEL: *value = struct_for_kernel(); return AT_OK;
    case AT_OPTION_BATCH_WAVES: *value = batch_waves(); return AT_OK;
    case AT_OPTION_G2P_BINS: *value = en.g2p_bins ? 1 : 0; return AT_OK;
    case AT_OPTION_BIN_REUSE: *value = en.bin_reuse; return AT_OK;
    case AT_OPTION_FUSE_BATCH: *value = en.fuse_batch ? 1 : 0; return AT_OK;
    case AT_OPTION_GRAPHS: *value = en.graphs ? 1 : 0; return AT_OK;
    case AT_OPTION_GRAPHS_CACHED: *value = (int64_t)en.graph_cache.size(); return AT_OK;
    case AT_OPTION_ASYNC: *value = en.async ? 1 : 0; return AT_OK;
    case AT_OPTION_VARIANTS: *value = variant_mode(); return AT_OK;
    case AT_OPTION_VARIANTS_LOADED: *value = variants_loaded(); return AT_OK;
    case AT_OPTION_VERIFY_DEMOTED: *value = en.verify_demoted ? 1 : 0; return AT_OK;
    default: return fail(AT_E_INVALID, "unknown option %d", option);
    }
}

at_status at_engine_reset(void) {
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    if (en.pipe) {
        std::lock_guard<std::mutex> pl(en.pipe->mu);
        en.pipe->err = AT_OK;
        en.pipe->msg.clear();
        en.pipe->sum = at_stats{};
    }
    en.persist = Persist{};
    en.cache.clear();
    en.queue.clear();
    drop_graphs(true);
    return AT_OK;
}

at_status at_ext_modified(const void *ptr) {
    if (!ptr) return fail(AT_E_INVALID, "null pointer");
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    en.persist.version[StateKey{(uint64_t)(uintptr_t)ptr, -1, ST_EXT}] += 1;
    return AT_OK;
}

// ----------------------------------------------------------------- batching

struct at_batch_s {
    at_batch_desc desc;
    BatchDev dev;
    size_t bytes;
    // admissions made through at_batch_update (host view)
    struct Grid {
        bool live = false;
        int32_t nb = 0;
        const int32_t *cells = nullptr;
        int32_t *slots = nullptr;
    };
    std::vector<Grid> grids;
    int32_t nfree = 0;       // height of the device free-slot stack
};

namespace {
struct BatchLayout {
    size_t clock, count, window, roots, work, rec, free_slots, x, xn, b, total;
};
at_status batch_layout(const at_batch_desc *d, BatchLayout &L, int32_t &R) {
    if (!d) return fail(AT_E_INVALID, "null batch description");
    if (d->reserved != 0) return fail(AT_E_INVALID, "reserved field must be 0");
    if (d->n <= 0 || d->n % kBS) return fail(AT_E_INVALID, "domain edge must be a positive multiple of 8");
    R = d->n / kBS;
    if ((int64_t)R * R * R > (1 << 20)) return fail(AT_E_INVALID, "batched grids are limited to R^3 <= 2^20 cells");
    if (d->max_grids < 1 || d->pool_blocks < 1) return fail(AT_E_INVALID, "max_grids and pool_blocks must be positive");
    if ((int64_t)d->max_grids * R * R * R >= (1LL << 31)) return fail(AT_E_INVALID, "max_grids * R^3 must fit in int32");
    const int64_t nc = (int64_t)R * R * R;
    size_t off = 0;
    L.clock = off; off += 128;
    L.count = off; off += 128;
    L.window = off; off += align256((size_t)d->max_grids * 2 * sizeof(int64_t));
    L.roots = off; off += align256((size_t)d->max_grids * nc * sizeof(int32_t));
    L.work = off; off += align256((size_t)d->pool_blocks * sizeof(int32_t));
    L.rec = off; off += align256((size_t)d->pool_blocks * 8 * sizeof(int32_t));
    L.free_slots = off; off += align256((size_t)d->pool_blocks * sizeof(int32_t));
    L.x = off; off += (size_t)d->pool_blocks * kBV * sizeof(float);
    L.xn = off; off += (size_t)d->pool_blocks * kBV * sizeof(float);
    L.b = off; off += (size_t)d->pool_blocks * kBV * sizeof(float);
    L.total = off;
    return AT_OK;
}
}  // namespace

at_status at_batch_footprint(const at_batch_desc *desc, size_t *bytes) {
    if (!bytes) return fail(AT_E_INVALID, "null output");
    BatchLayout L;
    int32_t R;
    at_status st = batch_layout(desc, L, R);
    if (st != AT_OK) return st;
    *bytes = L.total;
    return AT_OK;
}

at_status at_batch_create(const at_batch_desc *desc, void *dev_buf, size_t bytes, hipStream_t stream, at_batch *out) {
    if (!out) return fail(AT_E_INVALID, "null output handle");
    *out = nullptr;
    BatchLayout L;
    int32_t R;
    at_status st = batch_layout(desc, L, R);
    if (st != AT_OK) return st;
    if (!dev_buf || bytes < L.total) return fail(AT_E_INVALID, "batch buffer missing or below the footprint");
    if ((uintptr_t)dev_buf & 255) return fail(AT_E_INVALID, "batch buffer must be 256-byte aligned");
    char *b = (char *)dev_buf;
    at_batch h = new at_batch_s();
    h->desc = *desc;
    h->bytes = L.total;
    BatchDev &d = h->dev;
    d.R = R;
    d.R2 = R * R;
    d.ncells = R * R * R;
    d.max_grids = desc->max_grids;
    d.pool = desc->pool_blocks;
    d.clock = (int64_t *)(b + L.clock);
    d.count = (int32_t *)(b + L.count);
    d.window = (int64_t *)(b + L.window);
    d.roots = (int32_t *)(b + L.roots);
    d.work = (int32_t *)(b + L.work);
    d.rec = (int4 *)(b + L.rec);
    d.x = (float *)(b + L.x);
    d.xn = (float *)(b + L.xn);
    d.b = (float *)(b + L.b);
    d.free_slots = (int32_t *)(b + L.free_slots);
    h->grids.resize(desc->max_grids);
    h->nfree = desc->pool_blocks;
    hipError_t e = hipMemsetAsync(dev_buf, 0, L.total, stream);
    if (e == hipSuccess) e = hipMemsetAsync(d.roots, 0xff, (size_t)d.max_grids * d.ncells * sizeof(int32_t), stream);
    if (e == hipSuccess) e = launch_batch_init(d, stream);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "batch initialisation");
    }
    E().dispatches.fetch_add(3);
    *out = h;
    return AT_OK;
}

at_status at_batch_destroy(at_batch batch) {
    if (!batch) return fail(AT_E_INVALID, "null batch handle");
    delete batch;
    return AT_OK;
}

at_status at_batch_get_views(at_batch batch, at_batch_views *v) {
    if (!batch || !v) return fail(AT_E_INVALID, "null argument");
    const BatchDev &d = batch->dev;
    v->clock = d.clock;
    v->count = d.count;
    v->window = d.window;
    v->roots = d.roots;
    v->work = d.work;
    v->x = d.x;
    v->xn = d.xn;
    v->b = d.b;
    return AT_OK;
}

at_status at_batch_jacobi(at_batch batch, int32_t iters, int32_t workgroups, hipStream_t stream) {
    if (!batch) return fail(AT_E_INVALID, "null batch handle");
    if (iters < 0 || workgroups < 0) return fail(AT_E_INVALID, "negative iteration or workgroup count");
    if (iters == 0) return AT_OK;
    hipError_t e = launch_batch_jacobi(batch->dev, iters, workgroups, stream);
    if (e != hipSuccess) return hip_fail(e, "batched jacobi launch");
    E().dispatches.fetch_add(2 * (int64_t)iters + 2);
    return AT_OK;
}

at_status at_batch_update(at_batch batch, const at_batch_retire *retire, int32_t nretire, const at_batch_admit *admit,
                          int32_t nadmit, hipStream_t stream) {
    if (!batch) return fail(AT_E_INVALID, "null batch handle");
    if (nretire < 0 || nadmit < 0) return fail(AT_E_INVALID, "negative retirement or admission count");
    if ((nretire > 0 && !retire) || (nadmit > 0 && !admit)) return fail(AT_E_INVALID, "null descriptor array");
    const int32_t G = batch->desc.max_grids, pool = batch->desc.pool_blocks;
    auto &grids = batch->grids;
    // validate everything before anything is enqueued
    std::vector<char> out(G, 0), in(G, 0);
    int64_t freed = 0, taken = 0;
    for (int32_t r = 0; r < nretire; ++r) {
        const int32_t g = retire[r].gid;
        if (g < 0 || g >= G || !grids[g].live) return fail(AT_E_INVALID, "retirement %d: grid %d is not resident", r, g);
        if (out[g]) return fail(AT_E_INVALID, "grid %d retired twice in one update", g);
        if (retire[r].reserved != 0) return fail(AT_E_INVALID, "retirement %d: reserved field must be 0", r);
        out[g] = 1;
        freed += grids[g].nb;
    }
    for (int32_t a = 0; a < nadmit; ++a) {
        const at_batch_admit &A = admit[a];
        if (A.gid < 0 || A.gid >= G) return fail(AT_E_INVALID, "admission %d: grid id %d out of range", a, A.gid);
        if ((grids[A.gid].live && !out[A.gid]) || in[A.gid])
            return fail(AT_E_INVALID, "admission %d: grid %d is in use", a, A.gid);
        if (A.nblocks < 1 || A.nblocks > pool) return fail(AT_E_INVALID, "admission %d: %d blocks", a, A.nblocks);
        if (A.iters < 0) return fail(AT_E_INVALID, "admission %d: negative iteration count", a);
        if (!A.cells || !A.b || !A.slots) return fail(AT_E_INVALID, "admission %d: null device array", a);
        if (A.reserved != 0) return fail(AT_E_INVALID, "admission %d: reserved field must be 0", a);
        in[A.gid] = 1;
        taken += A.nblocks;
    }
    if (taken > (int64_t)batch->nfree + freed)
        return fail(AT_E_CAPACITY, "admissions need %lld pool blocks, %lld free", (long long)taken,
                    (long long)(batch->nfree + freed));
    const BatchDev &d = batch->dev;
    int64_t launches = 0;
    hipError_t e = hipSuccess;
    // retirements first: their slots go back on the stack, where the
    // admissions below may take them
    for (int32_t r0 = 0; r0 < nretire && e == hipSuccess; r0 += kUpdItems) {
        BatchRetireArgs ra{};
        for (int32_t r = r0; r < nretire && r < r0 + kUpdItems; ++r) {
            at_batch_s::Grid &gr = grids[retire[r].gid];
            BatchRetireItem &it = ra.it[ra.n++];
            it.gid = retire[r].gid;
            it.nb = gr.nb;
            it.q = batch->nfree;
            it.first = ra.blocks;
            it.cells = gr.cells;
            it.slots = gr.slots;
            it.x_out = retire[r].x_out;
            ra.blocks += gr.nb;
            batch->nfree += gr.nb;
            gr = at_batch_s::Grid{};
        }
        e = launch_batch_retire(d, ra, stream);
        ++launches;
    }
    for (int32_t a = 0; a < nadmit; ++a) {
        at_batch_s::Grid &gr = grids[admit[a].gid];
        gr.live = true;
        gr.nb = admit[a].nblocks;
        gr.cells = admit[a].cells;
        gr.slots = admit[a].slots;
    }
    // admissions, and the work list of every resident grid (ascending grid id)
    std::vector<BatchWorkItem> work;
    int32_t count = 0;
    for (int32_t g = 0; g < G; ++g)
        if (grids[g].live) {
            work.push_back(BatchWorkItem{g, grids[g].nb, count, 0, grids[g].cells});
            count += grids[g].nb;
        }
    const int64_t nl = std::max<int64_t>({(nadmit + kUpdItems - 1) / kUpdItems,
                                          ((int64_t)work.size() + kUpdGrids - 1) / kUpdGrids, (int64_t)1});
    for (int64_t l = 0; l < nl && e == hipSuccess; ++l) {
        BatchAdmitArgs aa{};
        aa.count = count;
        for (int32_t a = (int32_t)(l * kUpdItems); a < nadmit && a < (l + 1) * kUpdItems; ++a) {
            BatchAdmitItem &it = aa.it[aa.nadm++];
            it.gid = admit[a].gid;
            it.nb = admit[a].nblocks;
            batch->nfree -= it.nb;
            it.p = batch->nfree;
            it.first = aa.adm_blocks;
            it.iters = admit[a].iters;
            it.cells = admit[a].cells;
            it.b = admit[a].b;
            it.slots = admit[a].slots;
            aa.adm_blocks += it.nb;
        }
        for (size_t w = (size_t)(l * kUpdGrids); w < work.size() && w < (size_t)((l + 1) * kUpdGrids); ++w)
            aa.w[aa.nwork++] = work[w];
        e = launch_batch_admit(d, aa, stream);
        ++launches;
    }
    E().dispatches.fetch_add(launches);
    if (e != hipSuccess) return hip_fail(e, "batch update launch");
    return AT_OK;
}

int64_t at_dispatch_count(void) { return E().dispatches.load(); }

at_status at_timing_enable(int32_t on) {
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    en.timing = on != 0;
    return AT_OK;
}

at_status at_timing_collect(at_timing_entry *out, int32_t cap, int32_t *n) {
    if (cap < 0 || (cap > 0 && !out) || !n) return fail(AT_E_INVALID, "bad output array");
    Engine &en = E();
    std::lock_guard<std::recursive_mutex> lk(en.mu);
    drain_pipe(false);
    std::vector<at_timing_entry> acc;
    hipError_t err = hipSuccess;
    for (const Engine::Timed &t : en.timed) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess) {
            err = e;
        } else {
            size_t k = 0;
            while (k < acc.size() && !(acc[k].kind == t.kind && acc[k].op == t.op && acc[k].members == t.members)) ++k;
            if (k == acc.size()) acc.push_back(at_timing_entry{t.kind, t.op, t.members, 0, 0, 0.0});
            acc[k].launches += 1;
            acc[k].total_us += 1e3 * (double)ms;
        }
        en.ev_free.push_back(t.a);
        en.ev_free.push_back(t.b);
    }
    en.timed.clear();
    if (err != hipSuccess) return hip_fail(err, "timing events");
    const int32_t m = (int32_t)acc.size();
    *n = m < cap ? m : cap;
    for (int32_t i = 0; i < *n; ++i) out[i] = acc[i];
    if (m > cap) return fail(AT_E_CAPACITY, "%d timing entries, room for %d", m, cap);
    return AT_OK;
}

const char *at_last_error(void) { return g_err.c_str(); }

const char *at_version(void) { return "atsparse 0.1 (gfx950)"; }

}  // extern "C"
