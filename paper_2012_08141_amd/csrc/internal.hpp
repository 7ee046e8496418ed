// Internal definitions shared by the host runtime, the planner and the HIP
// kernels.  Not part of the public interface (include/atsparse.h is).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "atsparse.h"

namespace ats {

constexpr int kBS = 8;      // leaf block edge
constexpr int kBV = 512;    // voxels per leaf block

// Words of the per-grid device header (first 256 bytes of the grid buffer).
enum : int {
    HDR_COUNT = 0, HDR_BUMP = 1, HDR_ERR = 2, HDR_SCRATCH = 3, HDR_NBINS = 4, HDR_NAPPEND = 5,
    HDR_NOUT_ACC = 6,   // outliers listed so far by the scatter's first pass
    HDR_NOUT = 7        // outliers of the last binned scatter (pout[0..NOUT))
};
enum : int32_t { ERR_CAPACITY = 1, ERR_SPIN = 2, ERR_DEMOTED = 4 };

// Pointer-root cell states besides a valid slot (>= 0).
enum : int32_t { PTR_NULL = -1, PTR_LOCKED = -2, PTR_FAILED = -3 };

// Device view of one grid, passed by value to kernels.
struct GridDev {
    int32_t R;          // root edge (blocks per axis)
    int32_t R2;         // R * R
    int32_t kind;       // AT_ROOT_BITMASK / AT_ROOT_POINTER
    int32_t cap;        // leaf capacity (bitmask root: R^3)
    int64_t ncells;     // R^3
    uint32_t *bits;     // activity bits, one per root cell (both root kinds)
    int32_t *ptr;       // pointer root: slot per cell; bitmask root: nullptr
    int32_t *list;      // list state: records {cell, slot, 6 face-neighbour slots} (8 int32 each)
    int32_t *hdr;       // device header words
    float *chan;        // channel 0 base; channel c at chan + c * ch_stride
    int64_t ch_stride;  // floats per channel (cap * 512)
    uint64_t *scan;     // list generation look-back flags (kScanFlags entries)
    // particle binning workspace (absent when pcap == 0)
    int64_t pcap;       // particles that can be binned at once
    int32_t *pcount;    // [R^3] particles per root cell (zero between scatters)
    int32_t *poff;      // [R^3] first position of each cell's particles in pstage
    int4 *pbins;        // [R^3] non-empty cells: {cell, first, count, 0}; count in hdr[HDR_NBINS]
                        // (while ranking: cells appended in .x, count in hdr[HDR_NAPPEND])
    int2 *pkr;          // [pcap] per particle: {root cell of its centre node or -1, rank in that cell}
    float4 *pstage;     // [pcap][2] particle records {x0, x1, x2, v0}, {v1, v2, m, index} grouped by cell
    int32_t *pout;      // [pcap] particles whose centre node lies outside the domain (scattered directly)
};

constexpr int kScanFlags = 1024;   // = maximum workgroups of one list generation
constexpr int kRec = 8;            // int32 words per list record

// One op of a fused (or elementwise) struct-for program, applied per voxel
// in program order.
constexpr int kMaxOps = 16;
struct MicroOp {
    int32_t op;       // AT_OP_*
    int32_t ch[7];    // channels, as in the public op table
    float p;          // parameter
    uint32_t keep;    // FILL: bit q keeps the store to ch[q]; NORMALISE: bit c keeps v_c
    float p1;         // second parameter (ADVECT / MACCORMACK: 1 = RK3 back-trace; MPM_GRID: gravity)
    float p2;         // third parameter (MPM_GRID: wall thickness in nodes)
};
struct MicroProg {
    int32_t nops;
    int32_t check;    // eager activation check on writes
    int32_t table;    // neighbour slots from the list records (mask unchanged since listgen)
    int32_t verify;   // (no check) verify each listed block is still active; else flag ERR_DEMOTED, skip it
    MicroOp ops[kMaxOps];
};

// Particle program: any subset of gather (G2P), advection and scatter (P2G),
// in that order, over the same particle arrays.
enum : uint32_t { PS_G2P = 1, PS_ADVECT = 2, PS_P2G = 4 };
struct PartProg {
    uint32_t steps;
    int32_t act_mode;      // AT_ACT_* for the scatter
    int64_t np;
    float *x;              // [3][np], updated by ADVECT
    float *v;              // [3][np], written by G2P, read by ADVECT / P2G
    const float *m;        // [np]
    float dt;
    float inv_dx_src;      // gather grid
    float inv_dx_dst;      // scatter grid
    int32_t ch_vsrc;       // gather: velocity channels v0..v0+2 of gsrc
    int32_t ch_m, ch_mv;   // scatter: m and mv0..mv0+2 of gdst
    int32_t g2p_bins;      // gather through the bins in gbin_g (gsrc's last binned scatter had np particles)
    int32_t g2p_rec_x;     // and take positions from their records (they hold the current x)
    int32_t p2g_reuse;     // scatter over the bins in gbin_s as they are (no binning); the gather
                           // of the same node updates their records first
    GridDev gbin_g;        // workspace holding the bins the gather goes through
    GridDev gbin_s;        // workspace holding the bins the scatter uses (gdst unless reusing)
    GridDev gsrc, gdst;
};

// MLS-MPM particle program: any subset of gather (G2P_APIC), advection and
// scatter (P2G_MLS), in that order, over the same particle arrays, as one
// pass (the gathered v and C, and the advected x, reach the scatter in
// registers).
struct MpmProg {
    uint32_t steps;        // PS_G2P | PS_ADVECT | PS_P2G
    int32_t act_mode;      // AT_ACT_* for the scatter
    int64_t np;
    float *x;              // [3][np]
    float *v;              // [3][np]
    float *C;              // [9][np]
    float *F;              // [9][np]
    uint32_t keep;         // gather: bit 0 stores v, bit 1 stores C
    float adv_dt;          // advection
    float inv_dx_src;      // gather grid: 1 / dx
    float inv_dx_dst;      // scatter grid: 1 / dx
    float dt, mass, vol, mu, lam;   // scatter: F update and stress
    int32_t ch_vsrc;       // gather: v0..v0+2 of gsrc
    int32_t ch_m, ch_mv;   // scatter: m and mv0..mv0+2 of gdst
    GridDev gsrc, gdst;
};

// Batched Jacobi over many pointer-rooted grids sharing one leaf pool.
struct BatchDev {
    int32_t R, R2, ncells;   // per-grid root edge, R^2, R^3
    int32_t max_grids;
    int32_t pool;            // leaf pool size (blocks)
    int64_t *clock;          // global iteration counter
    int32_t *count;          // work list length
    int64_t *window;         // [max_grids][2]: first and one-past-last active iteration
    int32_t *roots;          // [max_grids][R^3]: pool slot or -1
    int32_t *work;           // [pool]: grid * R^3 + cell
    int4 *rec;               // [pool][2]: per work entry {slot, grid, nb0, nb1}, {nb2, nb3, nb4, nb5}
    float *x, *xn, *b;       // [pool][512]
    int32_t *free_slots;     // [pool]: stack of free pool slots (the host keeps its height)
};

// One batch update (at_batch_update) passes its descriptors by value, as
// kernel arguments: no host-to-device copy, nothing for the host to wait on.
constexpr int kUpdItems = 16;    // retirements or admissions per update launch
constexpr int kUpdGrids = 64;    // resident grids whose work entries one update launch writes
struct BatchRetireItem {
    int32_t gid, nb;
    int32_t q;                   // free-stack position its first slot is pushed to
    int32_t first;               // its first workgroup in the launch
    const int32_t *cells;        // [nb] root cells
    const int32_t *slots;        // [nb] pool slots (written by the admission)
    float *x_out;                // [nb][512] receives x, or null
};
struct BatchRetireArgs {
    int32_t n, blocks;
    BatchRetireItem it[kUpdItems];
};
struct BatchAdmitItem {
    int32_t gid, nb;
    int32_t p;                   // free-stack position of its first slot
    int32_t first;               // its first workgroup in the launch
    int32_t iters, pad;
    const int32_t *cells;        // [nb] root cells
    const float *b;              // [nb][512] right-hand side
    int32_t *slots;              // [nb] receives the pool slots
};
struct BatchWorkItem {
    int32_t gid, nb, off, pad;   // entries off .. off + nb - 1 of the work list
    const int32_t *cells;
};
struct BatchAdmitArgs {
    int32_t nadm, adm_blocks, nwork, count;
    BatchAdmitItem it[kUpdItems];
    BatchWorkItem w[kUpdGrids];
};

// Kernel launchers (kernels.hip).  Each enqueues exactly one dispatch on the
// stream and returns the launch status.
hipError_t launch_activate(const GridDev &g, const int32_t *ijk, int64_t n, int coord_kind,
                           hipStream_t s);
hipError_t launch_listgen(const GridDev &g, uint64_t *flags, uint32_t epoch, hipStream_t s);
hipError_t launch_stencil(const GridDev &g, int op, const int32_t *ch, float p, int check, int table,
                          hipStream_t s);
hipError_t launch_micro(const GridDev &g, const MicroProg &prog, hipStream_t s);
int wave_grid_size(const GridDev &g, bool pipelined);   // workgroups of the one-wavefront-per-block kernels

// A struct-for node of sampling ops (ADVECT, MACCORMACK) with element-wise
// ops beside them, run one workgroup of kTT threads per listed block with
// the block and a 2-voxel halo of every sampled channel staged in LDS.
constexpr int kTE = 12, kT3 = kTE * kTE * kTE;   // tile edge and voxels (block + 2 each side)
constexpr int kTileCh = 4;                        // sampled channels staged per node
constexpr int kTT = 512;                          // threads per workgroup
struct TileProg {
    MicroProg prog;
    int32_t nt;              // staged sampled channels
    int32_t tch[kTileCh];    // their grid channels
    int32_t vstage;          // stage the tile of v0 .. v0 + 2 (RK3 back-traces)
    int32_t v0;              // the velocity of every sampling op (else -1: read per voxel)
};
bool tile_prog(const MicroProg &prog, TileProg &tp);   // false: the node is not a tile program
size_t tile_lds_bytes(const TileProg &tp);             // dynamic LDS of one workgroup
unsigned tile_grid_size(const GridDev &g, size_t lds);  // workgroups of a tile launch

// Runtime-compiled variants of fused element-wise programs (jit.cpp).
// variant_launch: launches the program through its compiled variant when
// one is loaded (true; err has the launch status), else false (the caller
// runs the interpreter), queueing or doing the compilation per the mode.
bool variant_eligible(const MicroProg &prog);
bool variant_launch(const GridDev &g, const MicroProg &prog, hipStream_t s, hipError_t &err);
bool variant_prepare(const MicroProg &prog, int kind, std::string &src);   // generate and compile now (no device needed)
void set_variant_mode(int mode);   // 0 off, 1 compile in the background, 2 compile at first use
int variant_mode();
int64_t variants_loaded();
// A fused node whose first member is a single-output stencil op (LAP_UPDATE,
// JACOBI, DIFFUSE, channels ch) and whose other members are element-wise ops
// accepted by tail_op_supported (tail); neighbour slots from the list
// records, no activation check.
bool tail_op_supported(int op);
hipError_t launch_stencil_tail(const GridDev &g, int op, const int32_t *ch, float p, const MicroProg &tail,
                               hipStream_t s);
// Restriction (restrict_op; coarse[chc][I/2] += w * fine[chf][I]) or
// prolongation (fine[chf][I] += coarse[chc][I/2]) over the fine grid's list;
// check: activation on write of the blocks written; verify (without the
// check): a written block found inactive sets ERR_DEMOTED and is skipped.
hipError_t launch_transfer(bool restrict_op, const GridDev &f, const GridDev &c, int chf, int chc, float w,
                           int check, int verify, hipStream_t s);
// Launches one particle task (1 dispatch, or 4 when its scatter is binned;
// the count is stored in *dispatches).
hipError_t launch_particles(const PartProg &prog, hipStream_t s, int *dispatches);
// One MLS-MPM particle task (one dispatch).
hipError_t launch_mpm(const MpmProg &prog, hipStream_t s);
hipError_t launch_scatter_blocks(const GridDev &g, int ch, const int32_t *cells, const float *vals,
                                 int64_t n, hipStream_t s);
hipError_t launch_gather_blocks(const GridDev &g, int ch, const int32_t *cells, float *vals,
                                int64_t n, hipStream_t s);
hipError_t launch_popcount(const GridDev &g, hipStream_t s);   // into hdr[HDR_SCRATCH]
// iters x (jacobi, copy) over the work list, then clock += iters (2*iters + 1 dispatches).
hipError_t launch_batch_jacobi(const BatchDev &d, int iters, int workgroups, hipStream_t s);
hipError_t launch_batch_init(const BatchDev &d, hipStream_t s);
hipError_t launch_batch_retire(const BatchDev &d, const BatchRetireArgs &a, hipStream_t s);
hipError_t launch_batch_admit(const BatchDev &d, const BatchAdmitArgs &a, hipStream_t s);
int batch_waves();
void set_batch_waves(int waves);          // 1, 2 or 4 wavefronts per batched workgroup
// Binning workspace in the library's static device array (the scatter that
// allocates nothing): points g's workspace fields there and enqueues the
// clear of its counts (1 dispatch).  hipErrorInvalidValue when np or the
// grid's root cells exceed the array's limits.
constexpr int64_t kStaticParticles = AT_STATIC_MAX_PARTICLES;
constexpr int64_t kStaticCells = AT_STATIC_MAX_CELLS;
hipError_t static_bin_workspace(GridDev &g, int64_t np, hipStream_t s);
size_t static_workspace_bytes();
// Persistent grid size used by struct-for kernels (workgroups).
int struct_for_grid_size(const GridDev &g);
void set_struct_for_grid_size(int wgs);   // 0 = automatic
int struct_for_grid_size_override();       // the value set (0 = automatic)
int struct_for_kernel();
void set_struct_for_kernel(int form);     // 0 pipelined, 1 direct with records, 2 direct with root lookups

}  // namespace ats

// Host-side grid handle.
struct at_grid_s {
    at_grid_desc desc;
    ats::GridDev dev;
    uint64_t uid;       // engine identity (never reused)
    bool virt;          // planning handle without device memory
    uint32_t listgen_epoch;   // distinguishes list generation launches (never 0)
    size_t bytes;
    int32_t list_cap;
    // The last binned scatter into this grid: its particle count (0: none
    // since clear), position array, the window it ran in and the advections
    // of that array in the window up to it, and the grid whose workspace
    // holds its bins (this grid, or the source of a reused binning) with that
    // workspace's generation at the time.
    int64_t bins_np;
    const void *bins_x;
    uint64_t bins_window;
    int64_t bins_writes;
    uint64_t bins_owner;
    uint64_t bins_owner_gen;
    // This grid's own workspace: its generation (bumped when a scatter bins
    // into it and when the grid is cleared) and how many scatters have reused
    // its bins since they were made.
    uint64_t ws_gen;
    int32_t bins_age;
    float bins_inv_dx;      // 1/dx the particles were binned with
};
