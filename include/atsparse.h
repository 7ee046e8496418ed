/*
 * atsparse -- sparse-grid kernels with an inter-kernel optimizer, for
 * AMD Instinct MI355X (gfx950).
 *
 * The library implements the data-parallel hot path of the method of
 * "AsyncTaichi: On-the-fly Inter-kernel Optimizations for Imperative and
 * Spatially Sparse Programming" (Hu, Xu, Kuang, Durand; arXiv 2012.08141):
 * a spatially sparse grid (a bitmasked or pointer root over dense 8^3 fp32
 * leaf blocks, paper Section 3), the tasks that run on it (activation, list
 * generation, struct-for stencils, particle scatter and gather), and an
 * engine that runs a sequence of such tasks either eagerly or after the
 * paper's inter-kernel optimizations on a state-flow graph (Sections 4-7):
 * list generation removal, activation demotion, task fusion and dead store
 * elimination.
 *
 * Conventions for every entry point
 *   - Nothing throws across this interface.  Every call returns an
 *     at_status; on failure at_last_error() gives a message (thread-local,
 *     valid until the next failing call on the same thread).
 *   - An invalid argument returns AT_E_INVALID and enqueues no device work.
 *   - Device work is asynchronous on the hipStream_t passed in; the caller
 *     keeps every buffer alive until that work has completed.
 *   - The library never allocates device memory: the caller allocates each
 *     grid's buffer (size from at_grid_footprint) and every external array.
 *   - Layouts: a leaf block holds 512 fp32 values, voxel (i, j, k) of the
 *     block (local coordinates 0..7) at offset i*64 + j*8 + k.  Channels are
 *     stored structure-of-arrays: one array of capacity_blocks * 512 floats
 *     per channel.  The linear index of root cell (bi, bj, bk) is
 *     (bi*R + bj)*R + bk with R = n/8.  Particle arrays are SoA: x[3][np]
 *     (component c of particle p at c*np + p), v[3][np], m[np].
 *   - A grid handle is not thread-safe; the engine serialises its own state
 *     with a lock, so distinct handles may be used from distinct threads.
 */
#ifndef ATSPARSE_H
#define ATSPARSE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
typedef int32_t at_status;
#define AT_OK             0
#define AT_E_INVALID     -1   /* bad argument; nothing was enqueued */
#define AT_E_CAPACITY    -2   /* a grid's block pool ran out (sticky, see at_device_status) */
#define AT_E_HIP         -3   /* a HIP call failed; at_last_error() has its text */
#define AT_E_UNSUPPORTED -4   /* valid request the library does not implement */
#define AT_E_STATE       -5   /* call not allowed in the handle's current state */

/* ------------------------------------------------------------------- grids */
typedef struct at_grid_s *at_grid;

#define AT_ROOT_BITMASK 0   /* bitmasked root; every leaf preallocated, slot = cell */
#define AT_ROOT_POINTER 1   /* pointer root over a pool of capacity_blocks leaves */

typedef struct at_grid_desc {
    int32_t n[3];             /* domain edge in voxels per axis; multiples of 8, all equal */
    int32_t root_kind;        /* AT_ROOT_BITMASK or AT_ROOT_POINTER */
    int32_t channels;         /* fp32 value channels, 1..64 */
    int32_t capacity_blocks;  /* pointer root: pool size in leaves (<= R^3);
                                 bitmask root: ignored (R^3) */
    int32_t particle_capacity; /* particles a scatter into this grid may bin at
                                  once (workspace of 44 B each plus 24 B per root
                                  cell); a scatter of more particles, or any
                                  scatter when 0, adds straight into global
                                  memory with atomics instead of binning */
} at_grid_desc;

/* Bytes of device memory a grid with this description needs.  Host only.
 * (Section 3, "Spatially sparse programming": root, leaves, list.) */
at_status at_grid_footprint(const at_grid_desc *desc, size_t *bytes);

/* Create a grid in the caller's device buffer `dev_buf` of `bytes` bytes
 * (Section 3.2: a root over dense leaf blocks, every block inactive and
 * reading the ambient value 0 until activated; Section 4: the grid carries
 * the value, mask, list and allocator states the optimizer tracks).
 * `bytes` >= at_grid_footprint, 256-byte aligned.  Enqueues the buffer's
 * initialisation on `stream`: every block inactive, every value 0, empty
 * list.  The buffer stays owned by the caller and must outlive the handle.
 *
 * dev_buf == NULL (bytes ignored) creates a *planning handle*: it has no
 * device memory; at_run_sequence / at_plan_sequence accept it and plan and
 * record engine state for it but launch nothing, and every other call that
 * would touch device memory returns AT_E_STATE. */
at_status at_grid_create(const at_grid_desc *desc, void *dev_buf, size_t bytes,
                         hipStream_t stream, at_grid *out);

/* Release the host handle (the device buffer is the caller's).  Forgets the
 * engine's state-flow information for this grid: the states it owned leave
 * the graph, as the engine's garbage collection drops states nothing can
 * reach (Section 7.1).  Returns AT_E_INVALID for a NULL handle and
 * AT_E_STATE while tasks on the grid wait in the engine queue (flush first). */
at_status at_grid_destroy(at_grid grid);

/* Device pointers into the grid's buffer: where the value and list states
 * of Section 4 live, for callers that read or fill them directly (a write
 * through these pointers is invisible to the optimizer's state versions).
 * ch_base[c] (array of `channels`
 * entries, may be NULL) receives the base of channel c (capacity_blocks*512
 * floats, indexed by slot*512 + voxel).  *list receives the list state:
 * capacity min(R^3, capacity_blocks) records of 8 int32 -- root cell, leaf
 * slot, and the slots of the six face neighbours (i-1, i+1, j-1, j+1, k-1,
 * k+1; -1 inactive or outside) as of the list generation; *count its int32
 * length; *root the root table (bitmask root: uint32[ceil(R^3/32)] bits;
 * pointer root: int32[R^3] slot or -1).  Any out-pointer may be NULL. */
at_status at_grid_views(at_grid grid, float **ch_base, const int32_t **list,
                        const int32_t **count, const void **root);

typedef struct at_grid_info {
    int32_t n, R, root_kind, channels, capacity_blocks, list_capacity;
    int64_t ncells;           /* R^3 */
    size_t bytes;             /* footprint */
} at_grid_info;
at_status at_grid_get_info(at_grid grid, at_grid_info *info);

/* Deactivate every block: root emptied, used leaves zeroed, list emptied,
 * pool reset.  A deactivating write to the mask state (Section 4). */
at_status at_grid_clear(at_grid grid, hipStream_t stream);

/* Sticky device-side error bits of a grid, read synchronously on `stream`
 * (waits for the stream).  Activation allocates leaves from the grid's pool
 * (Section 3.2, pointer nodes); the pool's fixed capacity is this library's,
 * so running out is reported here instead of growing memory.  bit 0: the pointer pool overflowed
 * (AT_E_CAPACITY); bit 1: an allocation wait exceeded its spin limit; bit 2:
 * a write whose activation check was demoted found its block inactive
 * (only with AT_OPTION_VERIFY_DEMOTED).
 * Returns AT_OK and stores the bits; `clear` != 0 also resets them. */
at_status at_device_status(at_grid grid, hipStream_t stream, int32_t clear, int32_t *bits);

/* Number of active blocks (popcount of the mask), read synchronously. */
at_status at_active_count(at_grid grid, hipStream_t stream, int64_t *count);

/* -------------------------------------------------------- immediate tasks
 * Each call below runs one task eagerly (optimizer off) through the engine,
 * so the engine's state versions stay exact for later optimized windows. */

#define AT_COORD_VOXEL 0
#define AT_COORD_BLOCK 1

/* Activation on write (Section 3, item 3; Fig. 3): for each of the n
 * coordinates (device int32 [n][3]) activate the containing block.  A newly
 * activated block reads 0 in every channel; an active block is unchanged.
 * Coordinates outside the domain are ignored. */
at_status at_activate(at_grid grid, const int32_t *d_ijk, int64_t n, int32_t coord_kind,
                      hipStream_t stream);

/* List generation (Section 3, item 2): write the grid's list state -- a
 * record per active root cell, in ascending cell order, carrying the cell's
 * leaf slot and its face neighbours' slots -- and its device count.  The
 * list-clearing step is folded in (one dispatch). */
at_status at_listgen(at_grid grid, hipStream_t stream);

/* Struct-for operators over the grid's current list (Section 3, item 1).
 * Every voxel of every listed block is updated.  Neighbour reads outside
 * the domain or in inactive blocks give 0.  All arithmetic is fp32,
 * round-to-nearest, without contraction, in the order given:
 *   s = ((((x[i-1] + x[i+1]) + x[j-1]) + x[j+1]) + x[k-1]) + x[k+1]      */
#define AT_OP_LAP_UPDATE  1  /* ch {a, out}; p {coef}: out = a + coef*(s(a) - 6*a)        */
#define AT_OP_AXPY        2  /* ch {y, x};   p {alpha}: y = y + alpha*x                    */
#define AT_OP_JACOBI      3  /* ch {x, b, xn}: xn = (s(x) + b) * fp32(1/6)                 */
#define AT_OP_COPY        4  /* ch {dst, src}: dst = src                                   */
#define AT_OP_FILL        5  /* ch {c0, c1, ... , -1} (up to 7); p {value}: c = value       */
#define AT_OP_INC         6  /* ch {x}; p {value}: x = x + value                           */
#define AT_OP_DIFFUSE     7  /* ch {a, k, out}; p {dt}: per face q (same order as s),
                                kf = 0.5*(k + k_q); f = f + kf*(a_q - a); out = a + dt*f   */
#define AT_OP_DIFFUSE_ADJ 8  /* ch {a, k, lamn, lam, gk}; p {dt}: adjoint of DIFFUSE:
                                f = f + kf*(lamn_q - lamn); g = g + (a_q - a)*(lamn - lamn_q);
                                lam = lamn + dt*f; gk = gk + (dt*0.5)*g                    */
#define AT_OP_NORMALISE   9  /* ch {m, mv0, v0}: v_c = m > 0 ? mv_c / m : 0, c = 0..2 on
                                channels mv0+c, v0+c                                       */
#define AT_OP_ADVECT     10  /* ch {q, v0, out}; p {dt, rk3}: semi-Lagrangian advection
                                (the building block of the MacCormack benchmark, Section
                                8.2): out[I] = q at the back-traced point p (grid units; v
                                on channels v0..v0+2): p = I - dt*v(I) with rk3 = 0, or with
                                rk3 = 1 the RK3 back-trace v1 = v(I), p1 = I - (0.5dt)v1,
                                v2 = v(p1), p2 = I - (0.75dt)v2, v3 = v(p2),
                                p = I - dt*(2/9 v1 + 1/3 v2 + 4/9 v3) (v sampled like q);
                                q trilinear over the 8 voxels around p, corners
                                (a,b,c) lexicographic, weight (wx*wy)*wz, s = s + w*q;
                                reads outside the domain or in inactive blocks give 0; a
                                point more than 2 voxels outside is moved to 2 outside    */
#define AT_OP_MACCORMACK 11  /* ch {q, v0, fwd, bwd, out}; p {dt, rk3}: MacCormack
                                correction (Section 8.2): val = fwd + 0.5*(q - bwd)
                                (d = q - bwd, h = 0.5*d, val = fwd + h), clamped to the
                                range of q over the 8 corners around the back-traced point
                                of I (as for AT_OP_ADVECT; sparse reads; far points
                                moved as for AT_OP_ADVECT), fwd = ADVECT(q, dt) and
                                bwd = ADVECT(fwd, -dt)                                     */
#define AT_OP_MPM_GRID   12  /* ch {m, mv0, v0}; p {dt, g, bound}: the MLS-MPM grid
                                update (Section 8.3): where m > 0, v = mv / m, then
                                v_z = v_z - dt*g (z, axis 2, is up), then the walls: per
                                axis c, a voxel with index I_c < bound loses a negative v_c
                                and one with I_c > n - bound a positive v_c; where m == 0,
                                v = 0.  v may not overlap m or mv                           */

/* ch: host array of channel indices (meaning per op above); params: host
 * array of the op's parameters, in the order listed above (ADVECT and
 * MACCORMACK: 2, MPM_GRID: 3, the others 1; NULL for none).  check_activation != 0 keeps the per-write
 * activation check of an eager task (activation on write); 0 is the
 * demoted form (Section 6.3). */
at_status at_run_stencil(at_grid grid, int32_t op, const int32_t *ch, const float *params,
                         int32_t check_activation, hipStream_t stream);

/* Particle tasks (Section 8.3 workload; PIC transfers with the quadratic
 * B-spline: per axis base = floor(X - 0.5), fx = X - base,
 * w = (0.5*(1.5-fx)^2, 0.75-(fx-1)^2, 0.5*(fx-0.5)^2), X = x/dx, node weight
 * (wx*wy)*wz, nodes in (x, y, z) lexicographic order). */
#define AT_ACT_PER_NODE  0   /* eager: check and activate at each of the 27 node writes */
#define AT_ACT_PER_BLOCK 1   /* activate each distinct touched block once, then write unchecked */
#define AT_ACT_NONE      2   /* activate nothing: contributions to nodes of inactive blocks are
                                dropped (for callers that keep every touched block active) */

/* x += dt * v (device SoA arrays, np particles). */
at_status at_advect(float *d_x, const float *d_v, int64_t np, float dt, hipStream_t stream);

/* Scatter mass and momentum (Section 8.3's P2G, quadratic B-spline weights
 * w over the 27 nodes around each particle): m += w*m_p,
 * mv_c += (w*m_p)*v_c with fp32 atomics, activating node blocks on write.
 * ch: {m, mv0} (mv on mv0..mv0+2).  Nodes outside the domain are skipped.
 * When the grid's particle_capacity covers np, particles are first binned by
 * the block of their centre node and each bin is accumulated in an on-chip
 * tile (block plus halo) that is then added to the grid: five dispatches
 * instead of one, and the rounding of the fp32 sums differs (results agree
 * within the summation bound).  Binned scatters leave the bins in the grid's
 * workspace for later gathers from the grid (AT_OPTION_G2P_BINS) and fused
 * scatters of the same particles (AT_OPTION_BIN_REUSE). */
at_status at_p2g(at_grid grid, const float *d_x, const float *d_v, const float *d_m, int64_t np,
                 float dx, const int32_t *ch, int32_t activation, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): at_p2g that
 * always bins, through the library's own static binning workspace instead of
 * the grid's (so it also bins on grids created with particle_capacity 0).
 * Allocates nothing and calls no allocating routine; the workspace is one
 * file-scope device array of about 50 MiB per device, held until the process
 * ends.  Limits: np <= AT_STATIC_MAX_PARTICLES and R^3 <= AT_STATIC_MAX_CELLS
 * (a domain edge of at most 512), else AT_E_INVALID with nothing enqueued.
 * Same arguments, activation modes and result as at_p2g's binned scatter
 * (within the same summation bound); six dispatches: a clear of the
 * workspace's counts, then the five of the binned scatter.  Every call on a
 * device shares that device's workspace and leaves its contents behind:
 * calls that overlap on one device (on different streams, or from different
 * host threads without ordering) race and give wrong sums.  The bins are
 * not kept for later gathers or fused scatters (those use the grid's own
 * workspace). */
#define AT_STATIC_MAX_PARTICLES 1048576
#define AT_STATIC_MAX_CELLS     262144
at_status at_p2g_static(at_grid grid, const float *d_x, const float *d_v, const float *d_m, int64_t np,
                        float dx, const int32_t *ch, int32_t activation, hipStream_t stream);

/* Gather velocity (Section 8.3's G2P): v_p = sum over 27 nodes of w * v_node
 * (accumulated in node order from 0; 0 outside the domain or in inactive
 * blocks).  ch: {v0} (v on v0..v0+2).  After a binned scatter of as many
 * particles into this grid, the gather runs through those bins (one LDS tile
 * per bin) with bit-identical results. */
at_status at_g2p(at_grid grid, const float *d_x, float *d_v, int64_t np, float dx,
                 const int32_t *ch, hipStream_t stream);

/* MLS-MPM transfers (the falling cube of Section 8.3: moving least squares
 * MPM with APIC transfers and the fixed-corotated material).  Per-particle
 * state, all device SoA fp32: x, v [3][np]; C (affine velocity) and F
 * (deformation gradient) [9][np], row-major 3x3 per particle
 * (M_rc at M[(3r + c) * np + p]).  Weights, base and node order as for
 * at_p2g; fx = X - base per axis and the offset of node (a, b, d) from the
 * particle is dpos = ((a, b, d) - fx) * dx.
 *
 * Scatter: per particle F <- (I + dt C) F (stored), R the rotation of the
 * polar decomposition of F (Newton's iteration R <- (R + R^-T)/2 from F,
 * which needs det F > 0; fp32), J = det F, Kirchhoff stress
 * tau = 2 mu (F - R) F^T + lambda (J - 1) J I,
 * A = -(dt vol 4 / dx^2) tau + mass C; node (a, b, d) receives
 * m += w mass and mv += w (mass v + A dpos), with fp32 atomics in any order
 * (results agree with an in-order sum within the summation bound),
 * activating the blocks of the nodes written (AT_ACT_PER_NODE and
 * AT_ACT_PER_BLOCK activate the same blocks, once per block and
 * workgroup; AT_ACT_NONE drops contributions to inactive blocks).  Nodes
 * outside the domain are skipped.  ch: {m, mv0}.  Particles are processed in
 * chunks of 256 consecutive indices whose nodes are summed in an on-chip tile
 * first when they fit in 1,024 nodes (so spatially ordered particle arrays
 * scatter far faster; any order gives the same result). */
at_status at_p2g_mls(at_grid grid, const float *d_x, const float *d_v, const float *d_C, float *d_F,
                     int64_t np, float dx, float dt, float mass, float vol, float mu, float lambda,
                     const int32_t *ch, int32_t activation, hipStream_t stream);

/* Gather: v_p = sum of w v_node and C_p = (4 / dx^2) sum of w v_node dpos^T
 * over the 27 nodes, accumulated in node order from 0 as
 * wv = w * v_r; v_r = v_r + wv; B_rc = B_rc + wv * dpos_c, then C = (4/dx^2) B
 * (nodes outside the domain or in inactive blocks read 0).  ch: {v0}. */
at_status at_g2p_apic(at_grid grid, const float *d_x, float *d_v, float *d_C, int64_t np, float dx,
                      const int32_t *ch, hipStream_t stream);

/* Copy listed values between a grid and dense per-block arrays (setup and
 * inspection, not part of the optimized path).  cells: device int32 [n]
 * root cells; vals: device float [n][512].  at_scatter_blocks activates the
 * cells (in order) and stores; at_gather_blocks reads (0 for inactive). */
at_status at_scatter_blocks(at_grid grid, int32_t ch, const int32_t *d_cells, const float *d_vals,
                            int64_t n, hipStream_t stream);
at_status at_gather_blocks(at_grid grid, int32_t ch, const int32_t *d_cells, float *d_vals,
                           int64_t n, hipStream_t stream);

/* ---------------------------------------------------- sequences and engine
 * A task descriptor (Section 4, "Tasks"): the kind fixes the loop type
 * (serial, range-for or struct-for) and the states the task reads and
 * writes; the engine derives its state-flow edges from that.  Per kind:
 *   AT_TASK_ACTIVATE  range-for over n coordinates: grid; op = AT_COORD_*;
 *                     ext[0] = coords (int32 [n][3])
 *   AT_TASK_LISTGEN   serial: grid
 *   AT_TASK_STENCIL   struct-for over grid's list: op = AT_OP_*; ch = the op's
 *                     channels in the order documented there; param[0]
 *   AT_TASK_ADVECT    range-for over n particles: ext[0] = x (updated),
 *                     ext[1] = v; param[0] = dt
 *   AT_TASK_P2G       range-for: grid (scatter target); op = AT_ACT_* (the
 *                     eager form; the optimizer may coarsen it);
 *                     ext[0] = x, ext[1] = v, ext[2] = m; param[0] = dx;
 *                     ch[0] = m, ch[1] = mv0
 *   AT_TASK_G2P       range-for: grid (gather source); ext[0] = x,
 *                     ext[1] = v (written); param[0] = dx; ch[0] = v0
 *   AT_TASK_RESTRICT  struct-for over grid (the fine level); grid2 = the
 *                     coarse level (half the domain edge): for every listed
 *                     fine voxel I, coarse[ch[1]][I/2] += param[0] * fine[ch[0]][I],
 *                     activating the coarse blocks written (activation on
 *                     write).  The 8 children of a coarse voxel are added one
 *                     at a time in ascending order of their index inside
 *                     their (common) fine block.  The downsample pattern of
 *                     Section 6.3 (Fig. 5), in 3D.
 *   AT_TASK_PROLONG   struct-for over grid (fine); grid2 = coarse: for every
 *                     listed fine voxel I, fine[ch[1]][I] += coarse[ch[0]][I/2]
 *                     (an inactive coarse voxel reads 0; the coarse grid is
 *                     not written).  With RESTRICT, the transfers of the
 *                     multigrid solver of Section 8.4.
 *   AT_TASK_P2G_MLS   range-for: grid (scatter target); op = AT_ACT_*; the
 *                     MLS-MPM scatter of Section 8.3 (see at_p2g_mls):
 *                     ext[0] = x, ext[1] = v, ext[2] = C (read),
 *                     ext[3] = F (read and written); param = {dx, dt, mass,
 *                     vol, mu, lambda}; ch[0] = m, ch[1] = mv0
 *   AT_TASK_G2P_APIC  range-for: grid (gather source); the MLS-MPM gather
 *                     (see at_g2p_apic): ext[0] = x, ext[1] = v and
 *                     ext[2] = C (both written); param[0] = dx; ch[0] = v0.
 *                     With the loop_unique hint, G2P_APIC, ADVECT and
 *                     P2G_MLS over the same arrays fuse into one G2P2G task,
 *                     in which the gathered v and C reach the scatter in
 *                     registers, so dead store elimination can drop their
 *                     stores (supplement Section 4.4).
 * Unused ch entries must be -1 and unused ext entries NULL; grid2 is NULL
 * except for the two-level tasks. */
#define AT_TASK_ACTIVATE 1
#define AT_TASK_LISTGEN  2
#define AT_TASK_STENCIL  3
#define AT_TASK_ADVECT   4
#define AT_TASK_P2G      5
#define AT_TASK_G2P      6
#define AT_TASK_RESTRICT 7
#define AT_TASK_PROLONG  8
#define AT_TASK_P2G_MLS  9
#define AT_TASK_G2P_APIC 10

/* The particle arrays of this task are indexed only at the loop index, and
 * the loop index is unique per iteration and covers the array (the paper's
 * loop_unique hint, supplement Section 4.4).  Required for particle tasks
 * to be fusible. */
#define AT_TASKF_LOOP_UNIQUE 1u

typedef struct at_task {
    int32_t kind;         /* AT_TASK_* */
    int32_t op;           /* AT_OP_* (STENCIL), AT_COORD_* (ACTIVATE), AT_ACT_* (P2G) */
    uint32_t flags;       /* AT_TASKF_* */
    int32_t reserved;     /* must be 0 */
    at_grid grid;
    at_grid grid2;        /* coarse level of RESTRICT / PROLONG; NULL otherwise */
    int32_t ch[8];        /* channels; unused entries -1 */
    float param[8];       /* scalar parameters; unused entries 0 */
    void *ext[4];         /* device pointers of external arrays */
    int64_t n;            /* element count of a range-for (coordinates, particles) */
} at_task;

/* Optimizer passes (Section 6), selectable one by one as in the paper's
 * ablations.  0 = the eager pipeline. */
#define AT_OPT_LGR   1u   /* list generation removal (6.2) */
#define AT_OPT_AD    2u   /* activation demotion (6.3)     */
#define AT_OPT_FUSE  4u   /* task fusion (6.4, supplement 2) */
#define AT_OPT_DSE   8u   /* dead store elimination (6.5) */
#define AT_OPT_ALL  15u

typedef struct at_stats {
    int64_t tasks_in;             /* descriptors received */
    int64_t tasks_launched;       /* tasks left after optimization (fused = 1) */
    int64_t dispatches;           /* device dispatches issued (kernels + fills) */
    int64_t listgens_removed;
    int64_t activations_demoted;
    int64_t fusions;
    int64_t stores_eliminated;
    int64_t plan_cache_hits;
    double optimizer_us;          /* host time spent building and optimizing the plan */
} at_stats;

/* Run a window of tasks on `stream` (Section 5, lazy and asynchronous kernel launches):
 * build the state-flow graph (Section 4) seeded with the state owners kept
 * from earlier windows (Section 7.1, "Partial SFG garbage collection"), run
 * the passes selected in opt_flags to a fixpoint, and launch the result in a
 * topological order, without host synchronisation.  Results equal those of
 * running the tasks in the given order (order independency, Section 4.2).
 * stats (nullable) is overwritten with this window's counters. */
at_status at_run_sequence(const at_task *tasks, int32_t ntasks, uint32_t opt_flags,
                          at_stats *stats, hipStream_t stream);

/* One entry of an optimized plan: the input tasks it runs, in order. */
#define AT_PLAN_MAX_MEMBERS 16   /* = the most tasks one fused launch runs */
typedef struct at_plan_entry {
    int32_t kind;                 /* AT_TASK_* of the first member */
    int32_t nmembers;
    int32_t members[AT_PLAN_MAX_MEMBERS];   /* indices into the input task array */
    int32_t check_activation;     /* 1 if activating writes keep their check */
    int32_t activation_mode;      /* AT_ACT_* for particle scatter */
    uint32_t dropped;             /* bit q: member q lost some stores to DSE */
    uint32_t keep[AT_PLAN_MAX_MEMBERS];   /* per member: FILL channel slots / NORMALISE
                                             components still stored (all ones otherwise) */
} at_plan_entry;

/* Plan a window without running it or changing engine state (host only). */
at_status at_plan_sequence(const at_task *tasks, int32_t ntasks, uint32_t opt_flags,
                           at_plan_entry *out, int32_t capacity, int32_t *nout, at_stats *stats);

/* Queue a task for the next flush (Section 7.1, execution queue); flushes by
 * itself every `flush_period` tasks (AT_OPTION_FLUSH_PERIOD) with the
 * engine's opt flags (AT_OPTION_OPT_FLAGS). */
at_status at_enqueue(const at_task *task, hipStream_t stream);
/* Optimize and launch every queued task (Section 7.1, "Flushing"). */
at_status at_flush(at_stats *stats, hipStream_t stream);

#define AT_OPTION_MAX_FUSE_PER_TASK 1   /* default 1 (supplement Section 2, criterion 4) */
#define AT_OPTION_FLUSH_PERIOD      2   /* default 0 = flush only explicitly */
#define AT_OPTION_OPT_FLAGS         3   /* flags for at_enqueue/at_flush, default AT_OPT_ALL */
#define AT_OPTION_PLAN_CACHE        4   /* 1 (default) caches optimized plans */
#define AT_OPTION_STRUCT_FOR_WORKGROUPS 5 /* persistent struct-for grid size; 0 = automatic */
/* Struct-for kernel form (a tuning knob; results are identical):
 * 0 (default) software-pipelined kernels reading the list records,
 * 1 one block per wave iteration reading the list records,
 * 2 one block per wave iteration with neighbour lookups in the root.
 * Records are only read when list generation left them current. */
#define AT_OPTION_STRUCT_FOR_KERNEL 6
/* Wavefronts per workgroup of the batched Jacobi launches: 1 (default), 2
 * or 4; each wavefront sweeps its own blocks (a tuning knob; results are
 * identical).  Read when at_batch_jacobi enqueues (or a graph captures). */
#define AT_OPTION_BATCH_WAVES 7
/* Gathers through scatter bins: 1 (default) or 0.  A G2P whose source
 * grid's last binned scatter (since the grid was created or cleared) had the
 * same particle count gathers per bin from an LDS tile instead of per
 * particle from the grid; results are bit-identical either way.  A fused
 * node whose gather goes through bins runs its other steps (advection,
 * scatter) as one more dispatch in particle order.  Read when a node
 * executes. */
#define AT_OPTION_G2P_BINS 8
/* Bin reuse: how many scatters may reuse one binning of the particles
 * before they are binned again (default 8; 0 bins every scatter).  A node
 * that gathers through bins whose records hold the current positions,
 * advects and scatters into another grid of the same shape scatters over
 * those bins as they are: its gather first writes the new positions and
 * velocities into the records, and particles that have moved to a node next
 * to their bin's block are still summed in its tile (others scatter
 * directly).  Three dispatches instead of six; results agree within fp32
 * rounding of the scatter's sums.  Read when a node executes. */
#define AT_OPTION_BIN_REUSE 9
/* Fusion search: 1 (default) lets one simulation of the state-flow graph
 * serve several fusions where that provably gives the plan that fusing one
 * pair at a time (0) gives; the plans are the same, only planning time
 * differs.  Clears the plan cache. */
#define AT_OPTION_FUSE_BATCH 10
/* HIP graphs: 1 captures a window whose plan came from the plan cache,
 * which launches at least 16 nodes and which holds only struct-fors and
 * two-level transfers (no list generation, activation or particle task) into
 * a HIP graph on an internal stream the first time, and replays it on the
 * window's stream afterwards (default 0: launches are issued directly);
 * same launches, same results, one host call.  Cached graphs are dropped
 * when a grid they use is destroyed and on at_engine_reset. */
#define AT_OPTION_GRAPHS 11
/* Read-only: the number of window graphs currently cached. */
#define AT_OPTION_GRAPHS_CACHED 12
/* Asynchronous flushes (Section 7: the engine's optimizer and launcher run
 * beside the program): 1 hands every flushed window (at_flush, a periodic
 * flush, at_run_sequence) to an optimizer thread, which plans the windows in
 * flush order, and from it to a launcher thread, which launches them on
 * their streams; the call returns once the window is queued, so the
 * optimizer plans window k + 1 while window k is being launched and the
 * caller goes on enqueueing.  Default 0 (planned and launched inside the
 * call).  Plans, launches and results are those of the synchronous engine.
 * While windows are in flight every other engine call (activation, list
 * generation, grid creation and destruction, status reads, options, ...)
 * first waits until they have all been launched.  at_engine_sync waits
 * too and reports a failure of an asynchronous window; a failed window
 * drops the windows after it until the failure is reported.  The stats a
 * flush or at_run_sequence returns hold only tasks_in; at_engine_sync
 * returns the counters summed over the windows launched since the last
 * sync.  Launches happen on the launcher thread, with the device that was
 * current when the window was flushed; a device synchronisation waits only
 * for work launched, so call at_engine_sync first. */
#define AT_OPTION_ASYNC 13
/* Runtime-compiled variants (Sections 5 and 7.2: fused kernels compiled in
 * parallel with the program and kept in a cache): a fused struct-for of two
 * or more COPY, AXPY, INC, FILL and NORMALISE ops with no activation check
 * runs a kernel generated for its exact op sequence, compiled with hiprtc
 * for gfx950 and kept in memory and in $XDG_CACHE_HOME/atsparse/variants
 * (else ~/.cache/atsparse/variants), instead of the per-voxel interpreter.
 * It loads each channel it reads before writing once per block (the next
 * block's loads issued before this block's stores), keeps every value in
 * registers from op to op and stores each written channel once: same
 * results, bit for bit.  A node gets a variant only when that saves memory
 * traffic (the interpreter's per-voxel accesses at least 1.5 times the
 * variant's); others run the interpreter.  A node of semi-Lagrangian or
 * MacCormack ops (Section 8.2) with element-wise ops beside them, which runs
 * one workgroup per block over an LDS tile of the block and its 2-voxel
 * halo, gets a variant with its ops written out in place of the tile
 * kernel's op interpreter: same staging and arithmetic, same results bit
 * for bit.  0 (default): off; 1:
 * the first use queues the compilation on a worker thread and the node runs
 * the interpreter until the variant is loaded; 2: the first use compiles
 * (or reads the disk cache) before launching.  At most 256 variants. */
#define AT_OPTION_VARIANTS 14
/* Read-only: variants loaded on a device so far. */
#define AT_OPTION_VARIANTS_LOADED 15
/* Debug mode for activation demotion (Section 6.3): 1 makes every launched
 * node whose activating writes the optimizer demoted verify them: a
 * struct-for (run in the general interpreter, not the faster forms) checks
 * that each listed block is still active, and a restriction or
 * prolongation that each block it writes is active.  A block that is not
 * is skipped and sets bit 2 of the grid's sticky status (at_device_status).
 * A correct plan never sets it; the bit reports a demotion that was wrong,
 * or a mask changed behind the engine's back.  Default 0. */
#define AT_OPTION_VERIFY_DEMOTED 16
at_status at_set_option(int32_t option, int64_t value);
at_status at_get_option(int32_t option, int64_t *value);

/* Forget all engine state (versions, owners, cached plans). */
at_status at_engine_reset(void);

/* Generates and compiles, ahead of any launch, the variant
 * (AT_OPTION_VARIANTS) of a fused struct-for made of `tasks` in order (2 ..
 * 16 struct-for tasks of one grid, all stores kept), storing it in the
 * cache; no device is needed.  src (cap bytes, nullable when cap is 0)
 * receives the generated source, NUL-terminated and truncated to cap - 1,
 * and len (nullable) its full length.  AT_E_UNSUPPORTED when the program is
 * neither an element-wise chain whose variant saves memory traffic nor an
 * advection tile program, or the compilation failed; AT_E_INVALID for bad
 * tasks. */
at_status at_variant_prepare(const at_task *tasks, int32_t ntasks, char *src, size_t cap, size_t *len);

/* Waits until every window flushed asynchronously (AT_OPTION_ASYNC) has
 * been launched; stats (nullable) receives the counters summed over the
 * windows launched since the last sync.  Returns the first failure of such
 * a window since it was last reported (then cleared), else AT_OK.  A no-op
 * returning AT_OK when nothing was flushed asynchronously. */
at_status at_engine_sync(at_stats *stats);

/* Tell the engine an external array was written outside its tasks (bumps
 * the array's state version so no earlier result is reused). */
at_status at_ext_modified(const void *ptr);

/* ------------------------------------------------------------- batching
 * Many independent Jacobi solves (the 7-point Jacobi sweep and copy of
 * AT_OP_JACOBI / AT_OP_COPY, same arithmetic) over pointer-rooted grids of
 * one domain size whose leaves share one pool.  The caller owns admission:
 * it writes each grid's root row (pool slot per root cell, -1 inactive), its
 * pool leaves (x, b), the work list (entries grid * R^3 + cell, count) and
 * the grid's iteration window [start, end) in global iterations, through the
 * device views below, on the same stream.  at_batch_jacobi advances every
 * listed block whose grid is active at global iteration clock + i, for
 * i = 0 .. iters-1, then adds iters to the device clock.  Because all
 * per-launch state lives in device memory, the launches of one call can be
 * captured once in a HIP graph and replayed while grids come and go. */
typedef struct at_batch_s *at_batch;

typedef struct at_batch_desc {
    int32_t n;            /* domain edge of every grid (multiple of 8, R^3 <= 2^20) */
    int32_t max_grids;    /* grids that can be resident at once */
    int32_t pool_blocks;  /* shared leaf pool size */
    int32_t reserved;     /* must be 0 */
} at_batch_desc;

typedef struct at_batch_views {
    int64_t *clock;       /* global iteration counter (device) */
    int32_t *count;       /* work list length (device) */
    int64_t *window;      /* [max_grids][2] first and one-past-last active iteration */
    int32_t *roots;       /* [max_grids][R^3] pool slot or -1 */
    int32_t *work;        /* [pool_blocks] grid * R^3 + cell */
    float *x, *xn, *b;    /* [pool_blocks][512] */
} at_batch_views;

at_status at_batch_footprint(const at_batch_desc *desc, size_t *bytes);
/* Lays the batch out in the caller's buffer and enqueues its initialisation
 * (clock 0, empty work list, all windows empty, roots -1, pool zero). */
at_status at_batch_create(const at_batch_desc *desc, void *dev_buf, size_t bytes, hipStream_t stream,
                          at_batch *out);
at_status at_batch_destroy(at_batch batch);
at_status at_batch_get_views(at_batch batch, at_batch_views *views);
/* One pass that records, per work-list entry, its block's pool slot and the
 * slots of its six face neighbours (from the roots as they are now), then
 * iters x (jacobi, copy), then the clock tick: 2*iters + 2 dispatches, no
 * host synchronisation, no fills (safe to capture in a graph).  workgroups:
 * persistent grid size (0 = automatic).  The work list must hold at most
 * pool_blocks entries, each naming a grid below max_grids and a cell below
 * R^3, and the slots in the roots must lie below pool_blocks: the device
 * cannot check these.  An entry whose root cell holds no block is skipped. */
at_status at_batch_jacobi(at_batch batch, int32_t iters, int32_t workgroups, hipStream_t stream);

/* Library-managed admission and retirement for continuous batching (Section
 * 7.1: the host enqueues and goes on while the device computes).  One call
 * applies a replay boundary's changes in stream order: the retirements (each
 * grid's x copied out when x_out is given, its pool slots returned, its root
 * cells and window cleared), then the admissions (pool slots taken, b copied
 * in, x and xn zeroed, the root cells pointed at the slots, the window set
 * to [clock, clock + iters) from the device clock as it is when the update
 * runs, i.e. after every launch enqueued before it), then the work list of
 * every resident grid, in ascending grid id and each grid's cell order.
 * The descriptors travel as kernel arguments: no host-to-device copy and no
 * host synchronisation; 1 + ceil(nretire / 16) dispatches or more (one per
 * 16 admissions or 64 resident grids).  The pool's free slots are a stack
 * in device memory whose height the library tracks on the host.
 * Ownership: cells ([nblocks] root cells, distinct, below R^3), b
 * ([nblocks][512], block i for cells[i]) and slots ([nblocks], receives the
 * grid's pool slots) are caller device arrays; cells and slots must stay
 * valid until the grid is retired, b until the update has run; x_out
 * ([nblocks][512], block i for cells[i]) until the update has run.
 * Errors (nothing enqueued, state unchanged): AT_E_INVALID for a grid id
 * out of range, retiring a grid that is not resident (or twice), admitting
 * into a resident grid id (one retired in the same call may be reused),
 * nblocks outside [1, pool_blocks], negative iters or null arrays;
 * AT_E_CAPACITY when the admissions need more pool blocks than are free
 * after the retirements.  Cells outside the root cannot be checked on the
 * host: the device leaves them out of the roots and the sweep.  Grids made
 * this way must not also be written through the views (root rows, windows,
 * work list); reading x, xn and b through them is fine. */
typedef struct at_batch_admit {
    const int32_t *cells;
    const float *b;
    int32_t *slots;
    int32_t gid;          /* a grid id below max_grids that is not resident */
    int32_t nblocks;
    int32_t iters;        /* iterations the grid stays active */
    int32_t reserved;     /* must be 0 */
} at_batch_admit;

typedef struct at_batch_retire {
    int32_t gid;          /* a resident grid admitted through at_batch_update */
    int32_t reserved;     /* must be 0 */
    float *x_out;         /* nullable */
} at_batch_retire;

at_status at_batch_update(at_batch batch, const at_batch_retire *retire, int32_t nretire,
                          const at_batch_admit *admit, int32_t nadmit, hipStream_t stream);

/* Total device dispatches issued by the library since load. */
int64_t at_dispatch_count(void);

/* Per-launch timing of engine windows (a measurement aid).  While enabled,
 * every task the engine launches on a device grid is bracketed by a pair of
 * HIP events recorded on the window's stream (no host synchronisation).
 * at_timing_collect waits for the recorded events and returns, per launched
 * kind (task kind, op of its first member, number of fused members), the
 * launches and their total event-measured duration in microseconds, then
 * forgets them.  Events are created on first use and reused; out may be
 * NULL with cap 0 to discard.  Returns AT_E_CAPACITY (entries dropped) when
 * cap is too small. */
typedef struct at_timing_entry {
    int32_t kind, op, members, reserved;
    int64_t launches;
    double total_us;
} at_timing_entry;
at_status at_timing_enable(int32_t on);
at_status at_timing_collect(at_timing_entry *out, int32_t cap, int32_t *n);

/* Text of the last failing call on this thread (thread-local; valid until
 * the next failing call on the same thread; "" if none).  Not a step of the
 * paper's method: the error channel of a C interface that never throws. */
const char *at_last_error(void);
const char *at_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ATSPARSE_H */
