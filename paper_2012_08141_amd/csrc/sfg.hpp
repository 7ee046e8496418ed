// State-flow graph and inter-kernel optimizer (host C++, no device code).
//
// The paper's formulation (Section 4): a program is a sequence of tasks over
// states -- value states of fields, mask, list and allocator states of sparse
// nodes -- each state carrying a version bumped by every writer.  The union
// of the per-state writer chains with their reader branches is the
// state-flow graph (SFG), a DAG whose topological orders all give the same
// result.  Section 6 defines the passes run on it; here they operate on a
// task sequence kept in topological order, and every structural change is
// followed by a rebuild of the graph from that order (reconstruction
// invariance, Section 4.2).
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "internal.hpp"

namespace ats {

enum StKind : uint8_t { ST_VALUE = 0, ST_MASK = 1, ST_LIST = 2, ST_ALLOC = 3, ST_EXT = 4 };

struct StateKey {
    uint64_t obj;   // grid uid, or the address of an external array
    int32_t ch;     // value channel; -1 otherwise
    uint8_t kind;
    bool operator==(const StateKey &o) const { return obj == o.obj && ch == o.ch && kind == o.kind; }
};
struct StateKeyHash {
    size_t operator()(const StateKey &k) const;
};

enum : uint8_t { M_R = 1, M_W = 2 };
enum : uint8_t { P_ELEM = 0, P_STENCIL = 1, P_GATHER = 2, P_SCATTER = 3 };
enum : uint8_t { F_FULL = 1, F_ACTIVATING = 2, F_UNIQUE = 4 };

struct Access {
    StateKey s;
    uint8_t mode;      // M_R | M_W
    uint8_t pattern;   // P_*
    uint8_t flags;     // F_*
    int16_t member;    // index of the member task inside its node
};

enum LoopType : uint8_t { LT_SERIAL = 0, LT_RANGE = 1, LT_STRUCT = 2 };

struct Member {
    int32_t task;        // index into the window's task array
    uint32_t keep;       // FILL: channel slots kept; NORMALISE: components kept; else ~0
};

struct Node {
    std::vector<Member> members;   // in execution order
    bool check_activation = true;  // activating writes keep their check
    int32_t act_mode = AT_ACT_PER_NODE;
    // derived by derive():
    LoopType loop = LT_SERIAL;
    uint64_t loop_grid = 0;
    int64_t range = 0;
    std::vector<Access> acc;
};

// Engine state that survives a flush: state versions and what the latest
// owners of the list and mask states tell the next window (partial SFG
// garbage collection, Section 7.1).
struct Persist {
    std::unordered_map<StateKey, uint64_t, StateKeyHash> version;
    std::unordered_map<uint64_t, uint64_t> list_src;   // grid -> mask version its list was built from
    std::unordered_map<uint64_t, std::unordered_set<uint64_t>> act_sigs;  // grid -> activations done
    uint64_t ver(const StateKey &s) const {
        auto it = version.find(s);
        return it == version.end() ? 0 : it->second;
    }
    void forget_grid(uint64_t uid);
    void deactivate_grid(uint64_t uid);   // a deactivating write: clears owners' knowledge
};

struct PlanCounters {
    int64_t listgens_removed = 0, activations_demoted = 0, fusions = 0, stores_eliminated = 0;
};

// Look up the handle of a task's grid.
const at_grid_s *task_grid(const at_task &t);

// Validate a task descriptor; returns "" or an error message.
std::string validate_task(const at_task &t);

class Planner {
public:
    // batch_fusions: let one graph simulation serve several fusions where
    // that gives the same plan as fusing one pair at a time (false: one at
    // a time, the reference the batched planner is tested against)
    Planner(const at_task *tasks, int n, uint32_t flags, int max_fuse, bool batch_fusions = true);
    // Eager plan: one node per task, activation checks kept.
    void build_eager();
    // Run the selected passes to a fixpoint against `start`.
    void optimize(const Persist &start);
    // Apply the effects of executing `nodes` to the persistent state.
    static void commit(const std::vector<Node> &nodes, const at_task *tasks, Persist &p);
    // Predicate values the optimized plan depended on (for plan caching).
    static std::vector<uint8_t> fingerprint(const at_task *tasks, int n, const Persist &p);

    std::vector<Node> nodes;
    PlanCounters counters;

private:
    const at_task *tasks_;
    int n_;
    uint32_t flags_;
    int max_fuse_;
    bool batch_;
    bool pass_ad(const Persist &start);
    bool pass_lgr(const Persist &start);
    bool pass_dse(const Persist &start);
    bool pass_fuse_round(const Persist &start);
};

void derive(Node &nd, const at_task *tasks);
// For each node: 1 if it is a struct-for whose grid's mask is unchanged since
// its list was generated (the neighbour slots in the list records are valid).
std::vector<uint8_t> neighbour_tables_valid(const std::vector<Node> &nodes, const at_task *tasks, const Persist &p);
uint64_t hash_window(const at_task *tasks, int n, uint32_t flags, int max_fuse);

}  // namespace ats
