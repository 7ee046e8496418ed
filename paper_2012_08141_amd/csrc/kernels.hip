// HIP kernels of the sparse-grid hot path, written for gfx950 (CDNA4,
// 64-wide wavefronts).  Nothing here is a dense contraction, so nothing uses
// MFMA: the stencils are bandwidth-bound and are built around coalesced
// 16-byte block loads and an LDS block-plus-halo tile; list generation is a
// wavefront prefix-sum compaction; particle scatter uses fp32 atomics.
//
// Leaf layout: block slot s, voxel (i, j, k) at s*512 + i*64 + j*8 + k.  In
// every struct-for kernel thread t (of 128) owns the four voxels
// [4t, 4t+4) of the block -- row (i, j) = (t >> 4, (t >> 1) & 7), k from
// (t & 1) * 4 -- so each channel of a block moves as one 2 KiB fully
// coalesced dwordx4 access per wavefront pair.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace ats {
namespace {

constexpr int kSFThreads = 128;          // struct-for workgroup
int g_sf_grid_override = 0;
int g_sf_kernel = 0;
int g_batch_waves = 1;

#include "grid_device.hpp"

// Range of list entries a workgroup walks.  Workgroups are dispatched to the
// 8 XCDs round-robin; giving each XCD one contiguous slice of the (ascending)
// list keeps neighbouring blocks, whose faces are halo reads, in one L2.
struct ListRange {
    int lo, hi, step;
};
__device__ __forceinline__ ListRange list_range(int count) {
    const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
    const int x = blockIdx.x % nx;
    const int local = blockIdx.x / nx;
    const int per = gridDim.x / nx;
    const int lo = (int)(((int64_t)count * x) / nx);
    const int hi = (int)(((int64_t)count * (x + 1)) / nx);
    return {lo + local, hi, per};
}


__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// ------------------------------------------------------------- activation

template <int KIND>
__global__ __launch_bounds__(256) void k_activate(GridDev g, const int32_t *ijk, int64_t n, int coord_kind) {
    const int64_t N = (int64_t)g.R * kBS;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        int a = ijk[3 * t], b = ijk[3 * t + 1], c = ijk[3 * t + 2];
        if (coord_kind == AT_COORD_VOXEL) {
            if (a < 0 || b < 0 || c < 0 || a >= N || b >= N || c >= N) continue;
            a >>= 3; b >>= 3; c >>= 3;
        } else if (a < 0 || b < 0 || c < 0 || a >= g.R || b >= g.R || c >= g.R) {
            continue;
        }
        activate_cell<KIND>(g, ((int64_t)a * g.R + b) * g.R + c);
    }
}

// --------------------------------------------------------- list generation
// Workgroup b (256 threads) owns words [b*256*WPT, (b+1)*256*WPT) of the
// activity bits; thread t of it owns WPT consecutive words.  A block scan of
// per-thread popcounts gives offsets inside the workgroup; the workgroup's
// base offset comes from a single-pass decoupled look-back over its
// predecessors' published aggregates (flags[b] = epoch:32 | status:2 |
// value:30, status 1 = aggregate, 2 = inclusive prefix).  The host passes a
// fresh epoch per launch, so stale flags of an earlier launch are never
// mistaken for current ones and need no clearing.  Workgroups are
// dispatched in index order and every predecessor is resident or finished,
// so the bounded wait always ends.  The list comes out in ascending cell
// order; the last workgroup writes the count (the list clear is folded in).
constexpr int kScanMaxWG = 1024;
enum : uint32_t { SCAN_AGG = 1, SCAN_INCL = 2 };

__device__ __forceinline__ uint64_t scan_flag(uint32_t epoch, uint32_t status, uint32_t value) {
    return ((uint64_t)epoch << 32) | ((uint64_t)status << 30) | (uint64_t)value;
}

// Block record written for each list entry: the root cell, its leaf slot
// and the slots of its six face neighbours (order i-1, i+1, j-1, j+1, k-1,
// k+1; -1 when inactive or outside the domain), as of this list generation.
template <int KIND>
__device__ __forceinline__ int32_t lookup_slot(const GridDev &g, int64_t c, bool ok) {
    // unconditional load of a valid address; the select discards it
    const int64_t cc = ok ? c : 0;
    int32_t s;
    if (KIND == AT_ROOT_BITMASK) s = ((g.bits[cc >> 5] >> (cc & 31)) & 1u) ? (int32_t)cc : -1;
    else s = g.ptr[cc];
    return ok ? (s >= 0 ? s : -1) : -1;
}

template <int KIND>
__device__ __forceinline__ void write_record(const GridDev &g, int32_t cell, int pos) {
    int bi, bj, bk;
    cell_coords(g, cell, bi, bj, bk);
    const int32_t slot = (KIND == AT_ROOT_BITMASK) ? cell : g.ptr[cell];
    int4 *r = reinterpret_cast<int4 *>(g.list + (int64_t)pos * kRec);
    r[0] = make_int4(cell, slot, lookup_slot<KIND>(g, cell - g.R2, bi > 0), lookup_slot<KIND>(g, cell + g.R2, bi < g.R - 1));
    r[1] = make_int4(lookup_slot<KIND>(g, cell - g.R, bj > 0), lookup_slot<KIND>(g, cell + g.R, bj < g.R - 1),
                     lookup_slot<KIND>(g, cell - 1, bk > 0), lookup_slot<KIND>(g, cell + 1, bk < g.R - 1));
}

// Wave-parallel decoupled look-back: lane l inspects predecessor bid-1-l;
// the nearest predecessor with an inclusive prefix ends the walk, all
// nearer ones must have published their aggregate.  Bounded retries.
__device__ __forceinline__ int lookback(const GridDev &g, uint64_t *flags, uint32_t epoch, int bid) {
    const int lane = threadIdx.x & 63;
    int base = 0;
    int j = bid - 1;
    for (int it = 0; j >= 0;) {
        const int jj = j - lane;
        uint64_t f = scan_flag(epoch, SCAN_INCL, 0);    // before workgroup 0: prefix 0
        if (jj >= 0) f = __hip_atomic_load(&flags[jj], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t st = ((uint32_t)(f >> 32) == epoch) ? (uint32_t)(f >> 30) & 3u : 0u;
        const uint64_t incl = __ballot(st == SCAN_INCL);
        const uint64_t notready = __ballot(st == 0);
        const int L = incl ? __builtin_ctzll(incl) : 64;
        const uint64_t need = L == 64 ? ~0ull : ((2ull << L) - 1);
        if (notready & need) {
            if (++it >= kSpinLimit) {
                if (lane == 0) atomicOr(&g.hdr[HDR_ERR], ERR_SPIN);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        int v = lane <= L ? (int)(f & 0x3fffffffu) : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        base += v;
        if (L < 64) break;
        j -= 64;
    }
    return base;
}

// Thread t of workgroup b owns C consecutive root cells (C = 8 or 16: part
// of one bit word; C >= 32: C/32 whole words), so a dense run of active
// cells is spread over many threads and many workgroups.  For C <= 16 every
// lookup of a thread's records (its cells' slots and neighbour slots) is
// issued before any record is written.  With PREFIX (small roots: the bits
// before any workgroup's range are at most kPrefixWords words) each
// workgroup counts the active cells before its range itself, from the bits,
// instead of the look-back: no workgroup waits for another.
constexpr int64_t kPrefixWords = 8192;

template <int KIND, int C, bool PREFIX>
__global__ __launch_bounds__(256) void k_listgen(GridDev g, uint64_t *flags, uint32_t epoch) {
    constexpr int WPT = C >= 32 ? C / 32 : 1;
    __shared__ int wsum[4];
    __shared__ int wpre[4];
    __shared__ int s_base;
    const int64_t W = (g.ncells + 31) >> 5;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const uint32_t tail = (g.ncells & 31) ? ((1u << (g.ncells & 31)) - 1u) : 0xffffffffu;
    const int64_t c0 = ((int64_t)blockIdx.x * 256 + tid) * C;   // first cell of this thread
    uint32_t b[WPT];
    if (C < 32) {
        const int64_t w = c0 >> 5;
        uint32_t v = w < W ? g.bits[w] : 0u;
        if (w == W - 1) v &= tail;
        b[0] = (v >> (c0 & 31)) & ((1u << (C & 31)) - 1u);
    } else {
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int64_t w = (c0 >> 5) + q;
            uint32_t v = w < W ? g.bits[w] : 0u;
            if (w == W - 1) v &= tail;
            b[q] = v;
        }
    }
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < WPT; ++q) cnt += __popc(b[q]);
    // PREFIX: active cells in the (whole) words before this workgroup's range
    int pre = 0;
    if (PREFIX) {
        const int64_t wend = ((int64_t)blockIdx.x * 256 * C) >> 5;
        for (int64_t w = tid; w < wend; w += 256) pre += __popc(g.bits[w]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
        if (lane == 0) wpre[wid] = pre;
    }
    const int incl = wave_incl_scan(cnt);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    const int before = (wid > 0 ? wsum[0] : 0) + (wid > 1 ? wsum[1] : 0) + (wid > 2 ? wsum[2] : 0);
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (PREFIX) {
        if (tid == 0) {
            const int base = wpre[0] + wpre[1] + wpre[2] + wpre[3];
            s_base = base;
            if (blockIdx.x == gridDim.x - 1) g.hdr[HDR_COUNT] = base + total;
        }
    } else if (wid == 0) {
        const int bid = blockIdx.x;
        int base = 0;
        if (bid == 0) {
            if (lane == 0)
                __hip_atomic_store(&flags[0], scan_flag(epoch, SCAN_INCL, (uint32_t)total), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&flags[bid], scan_flag(epoch, SCAN_AGG, (uint32_t)total), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            base = lookback(g, flags, epoch, bid);
            if (lane == 0)
                __hip_atomic_store(&flags[bid], scan_flag(epoch, SCAN_INCL, (uint32_t)(base + total)),
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            s_base = base;
            if (bid == (int)gridDim.x - 1) g.hdr[HDR_COUNT] = base + total;
        }
    }
    __syncthreads();
    int pos = s_base + before + incl - cnt;
    if (C <= 16) {
        // all lookups first (C cells x 7), then the records
        int32_t sl[C], nb[C][6];
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int64_t cell = c0 + q;
            const bool on = (b[0] >> q) & 1u;
            const int64_t cc = on ? cell : 0;
            int bi, bj, bk;
            cell_coords(g, (int32_t)cc, bi, bj, bk);
            sl[q] = KIND == AT_ROOT_BITMASK ? (int32_t)cc : g.ptr[cc];
            nb[q][0] = lookup_slot<KIND>(g, cc - g.R2, on && bi > 0);
            nb[q][1] = lookup_slot<KIND>(g, cc + g.R2, on && bi < g.R - 1);
            nb[q][2] = lookup_slot<KIND>(g, cc - g.R, on && bj > 0);
            nb[q][3] = lookup_slot<KIND>(g, cc + g.R, on && bj < g.R - 1);
            nb[q][4] = lookup_slot<KIND>(g, cc - 1, on && bk > 0);
            nb[q][5] = lookup_slot<KIND>(g, cc + 1, on && bk < g.R - 1);
        }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            if (!((b[0] >> q) & 1u)) continue;
            int4 *r = reinterpret_cast<int4 *>(g.list + (int64_t)pos * kRec);
            r[0] = make_int4((int32_t)(c0 + q), sl[q], nb[q][0], nb[q][1]);
            r[1] = make_int4(nb[q][2], nb[q][3], nb[q][4], nb[q][5]);
            ++pos;
        }
    } else {
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            uint32_t v = b[q];
            const int64_t cb = c0 + 32 * q;
            while (v) {
                const int bit = __builtin_ctz(v);
                write_record<KIND>(g, (int32_t)(cb + bit), pos++);
                v &= v - 1;
            }
        }
    }
}

// ------------------------------------------------------ 7-point stencils
// One wavefront per block: lane l owns row (i, j) = (l >> 3, l & 7) of the
// block, i.e. the 8 consecutive voxels [8l, 8l+8) as two float4.  The i+-1
// and j+-1 neighbour rows are rows of the same block (lane +-8, +-1) or of
// the face-neighbour block; the k-1 / k+1 values beyond the row are single
// floats of the k-neighbour blocks.  Every lane issues all of its loads at
// once and unconditionally (an absent neighbour loads a valid dummy address
// and is zeroed by a select), so a block costs one dependent step (the six
// neighbour slots, looked up by lanes 0..5 and broadcast with readlane) plus
// one round of independent loads; there is no LDS and no barrier, and many
// small wavefronts per CU hide the latency.

struct StencilCh {
    const float *tin[3];  // stencil-read channels
    const float *ein;     // elementwise input (JACOBI: b; DIFFUSE_ADJ: gk)
    float *out0;          // output (LAP/DIFFUSE: out; JACOBI: xn; ADJ: lam)
    float *out1;          // DIFFUSE_ADJ: gk
};

template <int OP> struct NTiles { static constexpr int v = 1; };
template <> struct NTiles<AT_OP_DIFFUSE> { static constexpr int v = 2; };
template <> struct NTiles<AT_OP_DIFFUSE_ADJ> { static constexpr int v = 3; };

// Row values around a lane's 8 voxels: c[q] centre, f[face][q] the
// neighbour across `face` (order i-1, i+1, j-1, j+1, k-1, k+1).
struct Row {
    float c[8];
    float f[6][8];
};

__device__ __forceinline__ void put8(float *d, float4 a, float4 b) {
    d[0] = a.x; d[1] = a.y; d[2] = a.z; d[3] = a.w; d[4] = b.x; d[5] = b.y; d[6] = b.z; d[7] = b.w;
}

// Neighbour block slots of the wave's block, uniform across the wave.
struct Nbs {
    int32_t s[6];
};

template <int KIND>
__device__ __forceinline__ Nbs neighbour_slots(const GridDev &g, int32_t cell) {
    int bi, bj, bk;
    cell_coords(g, cell, bi, bj, bk);
    const int lane = threadIdx.x & 63;
    int32_t mine = -1;
    if (lane < 6) {
        bool ok;
        int64_t d;
        switch (lane) {
        case 0: ok = bi > 0; d = -(int64_t)g.R2; break;
        case 1: ok = bi < g.R - 1; d = g.R2; break;
        case 2: ok = bj > 0; d = -(int64_t)g.R; break;
        case 3: ok = bj < g.R - 1; d = g.R; break;
        case 4: ok = bk > 0; d = -1; break;
        default: ok = bk < g.R - 1; d = 1; break;
        }
        if (ok) mine = slot_of<KIND>(g, cell + d);
    }
    Nbs n;
#pragma unroll
    for (int f = 0; f < 6; ++f) n.s[f] = __builtin_amdgcn_readlane(mine, f);
    return n;
}

// Load the rows around this lane from channel `ch` (block slot `slot`).
__device__ __forceinline__ void load_row(const float *ch, int32_t slot, const Nbs &n, int lane, Row &r) {
    const int li = lane >> 3, lj = lane & 7;
    const int64_t own = (int64_t)slot * kBV;
    auto row_at = [&](bool inside, int in_row, int32_t nb, int nb_row, float *dst) {
        const bool present = inside || nb >= 0;
        const int64_t base = inside ? own + in_row * 8 : (nb >= 0 ? (int64_t)nb * kBV + nb_row * 8 : own);
        const float4 a = *reinterpret_cast<const float4 *>(ch + base);
        const float4 b = *reinterpret_cast<const float4 *>(ch + base + 4);
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        put8(dst, present ? a : z, present ? b : z);
    };
    {
        const float4 a = *reinterpret_cast<const float4 *>(ch + own + lane * 8);
        const float4 b = *reinterpret_cast<const float4 *>(ch + own + lane * 8 + 4);
        put8(r.c, a, b);
    }
    row_at(li > 0, lane - 8, n.s[0], lane + 56, r.f[0]);
    row_at(li < 7, lane + 8, n.s[1], lane - 56, r.f[1]);
    row_at(lj > 0, lane - 1, n.s[2], lane + 7, r.f[2]);
    row_at(lj < 7, lane + 1, n.s[3], lane - 7, r.f[3]);
    const float km = ch[(n.s[4] >= 0 ? (int64_t)n.s[4] * kBV : own) + lane * 8 + 7];
    const float kp = ch[(n.s[5] >= 0 ? (int64_t)n.s[5] * kBV : own) + lane * 8 + 0];
    r.f[4][0] = n.s[4] >= 0 ? km : 0.f;
    r.f[5][7] = n.s[5] >= 0 ? kp : 0.f;
#pragma unroll
    for (int q = 1; q < 8; ++q) r.f[4][q] = r.c[q - 1];
#pragma unroll
    for (int q = 0; q < 7; ++q) r.f[5][q] = r.c[q + 1];
}

__device__ __forceinline__ float nbsum(const Row &a, int q) {
    float s = a.f[0][q] + a.f[1][q];
    s = s + a.f[2][q];
    s = s + a.f[3][q];
    s = s + a.f[4][q];
    s = s + a.f[5][q];
    return s;
}

__device__ __forceinline__ void store8(float *d, const float *v) {
    reinterpret_cast<float4 *>(d)[0] = make_float4(v[0], v[1], v[2], v[3]);
    reinterpret_cast<float4 *>(d)[1] = make_float4(v[4], v[5], v[6], v[7]);
}

// The neighbour slots of a listed block: from its list record when the mask
// is known unchanged since the list was generated (TABLE), else looked up in
// the current root.
template <int KIND, bool TABLE>
__device__ __forceinline__ void read_record(const GridDev &g, int e, int32_t &cell, int32_t &slot, Nbs &n) {
    const int4 *r = reinterpret_cast<const int4 *>(g.list + (int64_t)e * kRec);
    const int4 a = r[0];
    cell = a.x;
    slot = a.y;
    if (TABLE) {
        const int4 b = r[1];
        n.s[0] = a.z; n.s[1] = a.w; n.s[2] = b.x; n.s[3] = b.y; n.s[4] = b.z; n.s[5] = b.w;
    } else {
        n = neighbour_slots<KIND>(g, cell);
    }
}

template <int OP, int KIND, bool CHECK, bool TABLE>
__global__ __launch_bounds__(64) void k_stencil(GridDev g, StencilCh c, float p) {
    const int lane = threadIdx.x;
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        int32_t cell, slot;
        Nbs n;
        read_record<KIND, TABLE>(g, e, cell, slot, n);
        int32_t wslot = slot;
        if (CHECK) {
            // activation on write of this block: one check per wavefront
            int32_t a = 0;
            if (lane == 0) a = activate_cell<KIND>(g, cell);
            wslot = __builtin_amdgcn_readfirstlane(a);
        }
        const int64_t off = (int64_t)wslot * kBV + lane * 8;
        const int64_t eoff = (int64_t)slot * kBV + lane * 8;
        float r0[8], r1[8];
        if (OP == AT_OP_LAP_UPDATE) {
            Row A;
            load_row(c.tin[0], slot, n, lane, A);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float s = nbsum(A, q);
                const float six_a = 6.0f * A.c[q];
                const float d = s - six_a;
                const float tq = p * d;
                r0[q] = A.c[q] + tq;
            }
            store8(c.out0 + off, r0);
        } else if (OP == AT_OP_JACOBI) {
            Row X;
            load_row(c.tin[0], slot, n, lane, X);
            float b[8];
            put8(b, reinterpret_cast<const float4 *>(c.ein + eoff)[0], reinterpret_cast<const float4 *>(c.ein + eoff)[1]);
            const float sixth = 0x1.555556p-3f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float s = nbsum(X, q);
                const float tq = s + b[q];
                r0[q] = tq * sixth;
            }
            store8(c.out0 + off, r0);
        } else if (OP == AT_OP_DIFFUSE) {
            Row A, K;
            load_row(c.tin[0], slot, n, lane, A);
            load_row(c.tin[1], slot, n, lane, K);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                float f = 0.f;
#pragma unroll
                for (int fc = 0; fc < 6; ++fc) {
                    const float kf = 0.5f * (K.c[q] + K.f[fc][q]);
                    f = f + kf * (A.f[fc][q] - A.c[q]);
                }
                r0[q] = A.c[q] + p * f;
            }
            store8(c.out0 + off, r0);
        } else if (OP == AT_OP_DIFFUSE_ADJ) {
            Row A, K, L;
            load_row(c.tin[0], slot, n, lane, A);
            load_row(c.tin[1], slot, n, lane, K);
            load_row(c.tin[2], slot, n, lane, L);
            float gk[8];
            put8(gk, reinterpret_cast<const float4 *>(c.ein + eoff)[0], reinterpret_cast<const float4 *>(c.ein + eoff)[1]);
            const float half_dt = p * 0.5f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                float f = 0.f, q2 = 0.f;
#pragma unroll
                for (int fc = 0; fc < 6; ++fc) {
                    const float kf = 0.5f * (K.c[q] + K.f[fc][q]);
                    f = f + kf * (L.f[fc][q] - L.c[q]);
                    q2 = q2 + (A.f[fc][q] - A.c[q]) * (L.c[q] - L.f[fc][q]);
                }
                r0[q] = L.c[q] + p * f;
                r1[q] = gk[q] + half_dt * q2;
            }
            store8(c.out0 + off, r0);
            store8(c.out1 + off, r1);
        }
    }
}

// ------------------------------------------- pipelined stencil (list table)
// When the list records' neighbour slots are valid (mask unchanged since the
// list generation), the stencil runs software-pipelined: the record of the
// next block comes through the scalar cache (the list is a read-only,
// non-aliased kernel argument) and all of that block's vector loads are
// issued before the current block's results are stored.  The loop body has
// no data-dependent branch (absent neighbours load a valid dummy address and
// are zeroed by a select), so the compiler can count outstanding loads
// exactly and never waits for the stores that follow them.

template <int NT, bool HAS_E>
struct Blk {
    int32_t slot;
    float4 c0[NT], c1[NT];                 // own row
    float4 f0[NT][4], f1[NT][4];           // i-1, i+1, j-1, j+1 rows
    float km[NT], kp[NT];                  // k-1 / k+1 beyond the row
    float4 e0, e1;                         // elementwise input
};

template <int NT, bool HAS_E>
__device__ __forceinline__ void fetch_blk(const StencilCh &c, const int32_t *__restrict__ recs, int e, int lane,
                                          Blk<NT, HAS_E> &B) {
    const int4 *r = reinterpret_cast<const int4 *>(recs + (int64_t)e * kRec);
    const int4 a = r[0], b = r[1];
    const int32_t slot = a.y;
    const int32_t nb[6] = {a.z, a.w, b.x, b.y, b.z, b.w};
    B.slot = slot;
    const int li = lane >> 3, lj = lane & 7;
    const int64_t own = (int64_t)slot * kBV;
    // row base of each of the 4 lateral neighbours (own block when inside)
    const bool in0 = li > 0, in1 = li < 7, in2 = lj > 0, in3 = lj < 7;
    int64_t base[4];
    base[0] = in0 ? own + (lane - 8) * 8 : (nb[0] >= 0 ? (int64_t)nb[0] * kBV + (lane + 56) * 8 : own);
    base[1] = in1 ? own + (lane + 8) * 8 : (nb[1] >= 0 ? (int64_t)nb[1] * kBV + (lane - 56) * 8 : own);
    base[2] = in2 ? own + (lane - 1) * 8 : (nb[2] >= 0 ? (int64_t)nb[2] * kBV + (lane + 7) * 8 : own);
    base[3] = in3 ? own + (lane + 1) * 8 : (nb[3] >= 0 ? (int64_t)nb[3] * kBV + (lane - 7) * 8 : own);
    const bool pr[4] = {in0 || nb[0] >= 0, in1 || nb[1] >= 0, in2 || nb[2] >= 0, in3 || nb[3] >= 0};
    const int64_t kmb = (nb[4] >= 0 ? (int64_t)nb[4] * kBV : own) + lane * 8 + 7;
    const int64_t kpb = (nb[5] >= 0 ? (int64_t)nb[5] * kBV : own) + lane * 8;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const float *ch = c.tin[nt];
        B.c0[nt] = *reinterpret_cast<const float4 *>(ch + own + lane * 8);
        B.c1[nt] = *reinterpret_cast<const float4 *>(ch + own + lane * 8 + 4);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const float4 u = *reinterpret_cast<const float4 *>(ch + base[f]);
            const float4 v = *reinterpret_cast<const float4 *>(ch + base[f] + 4);
            B.f0[nt][f] = pr[f] ? u : z;
            B.f1[nt][f] = pr[f] ? v : z;
        }
        const float km = ch[kmb], kp = ch[kpb];
        B.km[nt] = nb[4] >= 0 ? km : 0.f;
        B.kp[nt] = nb[5] >= 0 ? kp : 0.f;
    }
    if (HAS_E) {
        B.e0 = *reinterpret_cast<const float4 *>(c.ein + own + lane * 8);
        B.e1 = *reinterpret_cast<const float4 *>(c.ein + own + lane * 8 + 4);
    }
}

template <int NT, bool HAS_E>
__device__ __forceinline__ void unpack(const Blk<NT, HAS_E> &B, int nt, Row &r) {
    put8(r.c, B.c0[nt], B.c1[nt]);
#pragma unroll
    for (int f = 0; f < 4; ++f) put8(r.f[f], B.f0[nt][f], B.f1[nt][f]);
    r.f[4][0] = B.km[nt];
    r.f[5][7] = B.kp[nt];
#pragma unroll
    for (int q = 1; q < 8; ++q) r.f[4][q] = r.c[q - 1];
#pragma unroll
    for (int q = 0; q < 7; ++q) r.f[5][q] = r.c[q + 1];
}

// The values of a pipelined block for its op: r0 (and, for DIFFUSE_ADJ,
// r1) at the lane's 8 voxels; cin = the centre row of the first stencil
// input.
template <int OP, int NT, bool HAS_E>
__device__ __forceinline__ void pipe_compute(const Blk<NT, HAS_E> &cur, float p, float r0[8], float r1[8],
                                             float cin[8]) {
    put8(cin, cur.c0[0], cur.c1[0]);
    if (OP == AT_OP_LAP_UPDATE) {
        Row A;
        unpack(cur, 0, A);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float s = nbsum(A, q);
            const float six_a = 6.0f * A.c[q];
            const float d = s - six_a;
            const float tq = p * d;
            r0[q] = A.c[q] + tq;
        }
    } else if (OP == AT_OP_JACOBI) {
        Row X;
        unpack(cur, 0, X);
        float b[8];
        put8(b, cur.e0, cur.e1);
        const float sixth = 0x1.555556p-3f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float s = nbsum(X, q);
            const float tq = s + b[q];
            r0[q] = tq * sixth;
        }
    } else if (OP == AT_OP_DIFFUSE) {
        Row A, K;
        unpack(cur, 0, A);
        unpack(cur, 1, K);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            float f = 0.f;
#pragma unroll
            for (int fc = 0; fc < 6; ++fc) {
                const float kf = 0.5f * (K.c[q] + K.f[fc][q]);
                f = f + kf * (A.f[fc][q] - A.c[q]);
            }
            r0[q] = A.c[q] + p * f;
        }
    } else if (OP == AT_OP_DIFFUSE_ADJ) {
        Row A, K, L;
        unpack(cur, 0, A);
        unpack(cur, 1, K);
        unpack(cur, 2, L);
        float gk[8];
        put8(gk, cur.e0, cur.e1);
        const float half_dt = p * 0.5f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            float f = 0.f, q2 = 0.f;
#pragma unroll
            for (int fc = 0; fc < 6; ++fc) {
                const float kf = 0.5f * (K.c[q] + K.f[fc][q]);
                f = f + kf * (L.f[fc][q] - L.c[q]);
                q2 = q2 + (A.f[fc][q] - A.c[q]) * (L.c[q] - L.f[fc][q]);
            }
            r0[q] = L.c[q] + p * f;
            r1[q] = gk[q] + half_dt * q2;
        }
    }
}

template <int OP, int KIND, bool CHECK>
__global__ __launch_bounds__(64) void k_stencil_pipe(GridDev g, const int32_t *__restrict__ recs, StencilCh c,
                                                     float p) {
    constexpr int NT = NTiles<OP>::v;
    constexpr bool HAS_E = (OP == AT_OP_JACOBI || OP == AT_OP_DIFFUSE_ADJ);
    const int lane = threadIdx.x;
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    if (lr.lo >= lr.hi) return;
    Blk<NT, HAS_E> cur, nxt;
    fetch_blk<NT, HAS_E>(c, recs, __builtin_amdgcn_readfirstlane(lr.lo), lane, cur);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int en = e + lr.step < lr.hi ? e + lr.step : e;
        fetch_blk<NT, HAS_E>(c, recs, __builtin_amdgcn_readfirstlane(en), lane, nxt);
        int32_t wslot = cur.slot;
        if (CHECK) {
            const int32_t cell = recs[(int64_t)e * kRec];
            int32_t a = 0;
            if (lane == 0) a = activate_cell<KIND>(g, cell);
            wslot = __builtin_amdgcn_readfirstlane(a);
        }
        const int64_t off = (int64_t)wslot * kBV + lane * 8;
        float r0[8], r1[8];
        if (OP == AT_OP_LAP_UPDATE) {
            Row A;
            unpack(cur, 0, A);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float s = nbsum(A, q);
                const float six_a = 6.0f * A.c[q];
                const float d = s - six_a;
                const float tq = p * d;
                r0[q] = A.c[q] + tq;
            }
            store8(c.out0 + off, r0);
        } else if (OP == AT_OP_JACOBI) {
            Row X;
            unpack(cur, 0, X);
            float b[8];
            put8(b, cur.e0, cur.e1);
            const float sixth = 0x1.555556p-3f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float s = nbsum(X, q);
                const float tq = s + b[q];
                r0[q] = tq * sixth;
            }
            store8(c.out0 + off, r0);
        } else if (OP == AT_OP_DIFFUSE) {
            Row A, K;
            unpack(cur, 0, A);
            unpack(cur, 1, K);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                float f = 0.f;
#pragma unroll
                for (int fc = 0; fc < 6; ++fc) {
                    const float kf = 0.5f * (K.c[q] + K.f[fc][q]);
                    f = f + kf * (A.f[fc][q] - A.c[q]);
                }
                r0[q] = A.c[q] + p * f;
            }
            store8(c.out0 + off, r0);
        } else if (OP == AT_OP_DIFFUSE_ADJ) {
            Row A, K, L;
            unpack(cur, 0, A);
            unpack(cur, 1, K);
            unpack(cur, 2, L);
            float gk[8];
            put8(gk, cur.e0, cur.e1);
            const float half_dt = p * 0.5f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                float f = 0.f, q2 = 0.f;
#pragma unroll
                for (int fc = 0; fc < 6; ++fc) {
                    const float kf = 0.5f * (K.c[q] + K.f[fc][q]);
                    f = f + kf * (L.f[fc][q] - L.c[q]);
                    q2 = q2 + (A.f[fc][q] - A.c[q]) * (L.c[q] - L.f[fc][q]);
                }
                r0[q] = L.c[q] + p * f;
                r1[q] = gk[q] + half_dt * q2;
            }
            store8(c.out0 + off, r0);
            store8(c.out1 + off, r1);
        }
        cur = nxt;
    }
}

// ------------------------------------- pipelined stencil, LDS-staged rows
// The one-input ops (LAP_UPDATE, JACOBI) with the rows a lane needs from the
// rest of its block, and from the four lateral neighbour faces, taken from
// LDS instead of being loaded again through the vector memory path: per
// block and lane the loads are the own row (2 x 16 B), a quarter-row of one
// lateral neighbour face (16 B: lanes 16f .. 16f + 15 load face f), the two
// k-end values and, for JACOBI, b (2 x 16 B) -- 7 loads instead of 14.  The
// wave (one per workgroup) writes its block's rows and the faces to LDS,
// split into the first and second float4 of every row so that the 16-byte
// reads of 64 lanes fall on distinct banks, then reads the i -+ 1 and j -+ 1
// rows from there.  Software-pipelined as k_stencil_pipe: the next block's
// loads are in flight while the current block is computed; a wave-scope
// fence keeps the LDS writes and reads in program order across lanes (LDS
// operations of one wave execute in order).  Same values, same arithmetic.
constexpr bool kStencilLds = true;

template <bool HAS_E>
struct BlkL {
    int32_t slot;
    float4 c0, c1;       // own row
    float4 face;         // this lane's piece of a lateral face (zero when absent)
    float km, kp;        // k-1 / k+1 beyond the row
    float4 e0, e1;       // elementwise input
};

// Loads of one block from its record: a = {cell, slot, i-1, i+1}, b = {j-1,
// j+1, k-1, k+1} (neighbour slots, -1 when absent); slot must be valid.
template <bool HAS_E>
__device__ __forceinline__ void fetch_rec_lds(const StencilCh &c, const int4 a, const int4 b, int lane,
                                              BlkL<HAS_E> &B) {
    const int32_t slot = a.y;
    B.slot = slot;
    const int64_t own = (int64_t)slot * kBV;
    const float *ch = c.tin[0];
    B.c0 = *reinterpret_cast<const float4 *>(ch + own + lane * 8);
    B.c1 = *reinterpret_cast<const float4 *>(ch + own + lane * 8 + 4);
    // face f of the neighbour across it: i-1 (its plane i = 7), i+1 (i = 0),
    // j-1 (j = 7), j+1 (j = 0); piece q = 2 * row + half
    const int f = lane >> 4, q = lane & 15, row = q >> 1, h = q & 1;
    const int32_t nf = f == 0 ? a.z : f == 1 ? a.w : f == 2 ? b.x : b.y;
    const int fo = f == 0 ? 7 * 64 + row * 8 : f == 1 ? row * 8 : f == 2 ? row * 64 + 7 * 8 : row * 64;
    const float4 fv = *reinterpret_cast<const float4 *>(ch + (nf >= 0 ? (int64_t)nf * kBV : own) + fo + 4 * h);
    B.face = nf >= 0 ? fv : make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t kmb = (b.z >= 0 ? (int64_t)b.z * kBV : own) + lane * 8 + 7;
    const int64_t kpb = (b.w >= 0 ? (int64_t)b.w * kBV : own) + lane * 8;
    const float km = ch[kmb], kp = ch[kpb];
    B.km = b.z >= 0 ? km : 0.f;
    B.kp = b.w >= 0 ? kp : 0.f;
    if (HAS_E) {
        B.e0 = *reinterpret_cast<const float4 *>(c.ein + own + lane * 8);
        B.e1 = *reinterpret_cast<const float4 *>(c.ein + own + lane * 8 + 4);
    }
}

template <bool HAS_E>
__device__ __forceinline__ void fetch_blk_lds(const StencilCh &c, const int32_t *__restrict__ recs, int e, int lane,
                                              BlkL<HAS_E> &B) {
    const int4 *r = reinterpret_cast<const int4 *>(recs + (int64_t)e * kRec);
    fetch_rec_lds<HAS_E>(c, r[0], r[1], lane, B);
}

template <int OP, bool CHECK, int KIND>
__global__ __launch_bounds__(64) void k_stencil_lds(GridDev g, const int32_t *__restrict__ recs, StencilCh c, float p) {
    constexpr bool HAS_E = OP == AT_OP_JACOBI;
    __shared__ float4 s_own[2][64];       // [half][row]: float4 h of row (i, j) = lane
    __shared__ float4 s_face[2][4][8];    // [half][face][row]
    const int lane = threadIdx.x;
    const int li = lane >> 3, lj = lane & 7;
    const int f = lane >> 4, frow = (lane & 15) >> 1, fh = lane & 1;
    // LDS sources of this lane's i-1, i+1, j-1, j+1 rows: the own block's
    // row, or row lj (i faces) / li (j faces) of a face
    const float4 *src[4] = {li > 0 ? &s_own[0][lane - 8] : &s_face[0][0][lj],
                            li < 7 ? &s_own[0][lane + 8] : &s_face[0][1][lj],
                            lj > 0 ? &s_own[0][lane - 1] : &s_face[0][2][li],
                            lj < 7 ? &s_own[0][lane + 1] : &s_face[0][3][li]};
    const int hstride[4] = {li > 0 ? 64 : 32, li < 7 ? 64 : 32, lj > 0 ? 64 : 32, lj < 7 ? 64 : 32};
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    if (lr.lo >= lr.hi) return;
    BlkL<HAS_E> cur, nxt;
    fetch_blk_lds<HAS_E>(c, recs, __builtin_amdgcn_readfirstlane(lr.lo), lane, cur);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int en = e + lr.step < lr.hi ? e + lr.step : e;
        fetch_blk_lds<HAS_E>(c, recs, __builtin_amdgcn_readfirstlane(en), lane, nxt);
        int32_t wslot = cur.slot;
        if (CHECK) {
            const int32_t cell = recs[(int64_t)e * kRec];
            int32_t a = 0;
            if (lane == 0) a = activate_cell<KIND>(g, cell);
            wslot = __builtin_amdgcn_readfirstlane(a);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // the last block's reads come first
        s_own[0][lane] = cur.c0;
        s_own[1][lane] = cur.c1;
        s_face[fh][f][frow] = cur.face;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // then this block's writes
        Row X;
        put8(X.c, cur.c0, cur.c1);
#pragma unroll
        for (int d = 0; d < 4; ++d) put8(X.f[d], src[d][0], src[d][hstride[d]]);
        X.f[4][0] = cur.km;
        X.f[5][7] = cur.kp;
#pragma unroll
        for (int q = 1; q < 8; ++q) X.f[4][q] = X.c[q - 1];
#pragma unroll
        for (int q = 0; q < 7; ++q) X.f[5][q] = X.c[q + 1];
        const int64_t off = (int64_t)wslot * kBV + lane * 8;
        float r0[8];
        if (OP == AT_OP_LAP_UPDATE) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float sum = nbsum(X, q);
                const float six_a = 6.0f * X.c[q];
                const float d = sum - six_a;
                const float tq = p * d;
                r0[q] = X.c[q] + tq;
            }
        } else {
            float bb[8];
            put8(bb, cur.e0, cur.e1);
            const float sixth = 0x1.555556p-3f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float sum = nbsum(X, q);
                const float tq = sum + bb[q];
                r0[q] = tq * sixth;
            }
        }
        store8(c.out0 + off, r0);
        cur = nxt;
    }
}

// The element-wise tail of a fused stencil node, applied per voxel in
// program order to the lane's 8 voxels: the stencil's output (out_ch) stays
// in r0 until the caller stores it, the centre row of its first input
// (in_ch) is cin, other channels are read and written at the voxel.
__device__ __forceinline__ void apply_tail(const GridDev &g, const MicroProg &tail, int64_t off, int out_ch, int in_ch,
                                           float r0[8], float cin[8]) {
    auto get = [&](int ch, float v[8]) {
        if (ch == out_ch) {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = r0[q];
        } else if (ch == in_ch) {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = cin[q];
        } else {
            const float *src = chan(g, ch) + off;
            put8(v, reinterpret_cast<const float4 *>(src)[0], reinterpret_cast<const float4 *>(src)[1]);
        }
    };
    auto set = [&](int ch, const float v[8]) {
        if (ch == out_ch) {
#pragma unroll
            for (int q = 0; q < 8; ++q) r0[q] = v[q];
        } else {
            store8(chan(g, ch) + off, v);
            if (ch == in_ch) {
#pragma unroll
                for (int q = 0; q < 8; ++q) cin[q] = v[q];
            }
        }
    };
    for (int o = 0; o < tail.nops; ++o) {
        const MicroOp &op = tail.ops[o];
        float y[8], x[8];
        switch (op.op) {
        case AT_OP_AXPY:
            get(op.ch[0], y);
            get(op.ch[1], x);
#pragma unroll
            for (int q = 0; q < 8; ++q) y[q] = y[q] + op.p * x[q];
            set(op.ch[0], y);
            break;
        case AT_OP_INC:
            get(op.ch[0], y);
#pragma unroll
            for (int q = 0; q < 8; ++q) y[q] = y[q] + op.p;
            set(op.ch[0], y);
            break;
        case AT_OP_COPY:
            get(op.ch[1], y);
            set(op.ch[0], y);
            break;
        case AT_OP_FILL:
#pragma unroll
            for (int q = 0; q < 8; ++q) y[q] = op.p;
            for (int k = 0; k < 7; ++k)
                if (op.ch[k] >= 0 && ((op.keep >> k) & 1u)) set(op.ch[k], y);
            break;
        default:
            break;
        }
    }
}

// A fused struct-for whose first member is a single-output stencil op
// (LAP_UPDATE, JACOBI, DIFFUSE) followed by element-wise ops (AXPY, INC,
// COPY, FILL): the stencil runs pipelined as above and the element-wise ops
// are applied per voxel, in program order, to the lane's 8 voxels.  The
// stencil's output stays in registers until the end and the centre row of its
// first input is reused; other channels are read and written at the voxel
// (a thread sees its own earlier stores).  No activation check: fused nodes
// with one run the general interpreter.
template <int OP, int KIND>
__global__ __launch_bounds__(64) void k_stencil_tail(GridDev g, const int32_t *__restrict__ recs, StencilCh c,
                                                     float p, MicroProg tail, int out_ch, int in_ch) {
    constexpr int NT = NTiles<OP>::v;
    constexpr bool HAS_E = (OP == AT_OP_JACOBI || OP == AT_OP_DIFFUSE_ADJ);
    const int lane = threadIdx.x;
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    if (lr.lo >= lr.hi) return;
    Blk<NT, HAS_E> cur, nxt;
    fetch_blk<NT, HAS_E>(c, recs, __builtin_amdgcn_readfirstlane(lr.lo), lane, cur);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int en = e + lr.step < lr.hi ? e + lr.step : e;
        fetch_blk<NT, HAS_E>(c, recs, __builtin_amdgcn_readfirstlane(en), lane, nxt);
        const int64_t off = (int64_t)cur.slot * kBV + lane * 8;
        float r0[8], r1[8], cin[8];
        pipe_compute<OP, NT, HAS_E>(cur, p, r0, r1, cin);
        apply_tail(g, tail, off, out_ch, in_ch, r0, cin);
        store8(c.out0 + off, r0);
        cur = nxt;
    }
}

// The same for a Jacobi or lap_update head in the form of k_stencil_lds:
// the block's rows and lateral faces staged through LDS, the next block's
// loads issued before this block computes.  Same arithmetic, same results.
template <int OP>
__global__ __launch_bounds__(64) void k_stencil_tail_lds(GridDev g, const int32_t *__restrict__ recs, StencilCh c,
                                                         float p, MicroProg tail, int out_ch, int in_ch) {
    constexpr bool HAS_E = OP == AT_OP_JACOBI;
    __shared__ float4 s_own[2][64];
    __shared__ float4 s_face[2][4][8];
    const int lane = threadIdx.x;
    const int li = lane >> 3, lj = lane & 7;
    const int f = lane >> 4, frow = (lane & 15) >> 1, fh = lane & 1;
    const float4 *src[4] = {li > 0 ? &s_own[0][lane - 8] : &s_face[0][0][lj],
                            li < 7 ? &s_own[0][lane + 8] : &s_face[0][1][lj],
                            lj > 0 ? &s_own[0][lane - 1] : &s_face[0][2][li],
                            lj < 7 ? &s_own[0][lane + 1] : &s_face[0][3][li]};
    const int hstride[4] = {li > 0 ? 64 : 32, li < 7 ? 64 : 32, lj > 0 ? 64 : 32, lj < 7 ? 64 : 32};
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    if (lr.lo >= lr.hi) return;
    BlkL<HAS_E> cur, nxt;
    fetch_blk_lds<HAS_E>(c, recs, __builtin_amdgcn_readfirstlane(lr.lo), lane, cur);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int en = e + lr.step < lr.hi ? e + lr.step : e;
        fetch_blk_lds<HAS_E>(c, recs, __builtin_amdgcn_readfirstlane(en), lane, nxt);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // the last block's reads come first
        s_own[0][lane] = cur.c0;
        s_own[1][lane] = cur.c1;
        s_face[fh][f][frow] = cur.face;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // then this block's writes
        Row X;
        put8(X.c, cur.c0, cur.c1);
#pragma unroll
        for (int d = 0; d < 4; ++d) put8(X.f[d], src[d][0], src[d][hstride[d]]);
        X.f[4][0] = cur.km;
        X.f[5][7] = cur.kp;
#pragma unroll
        for (int q = 1; q < 8; ++q) X.f[4][q] = X.c[q - 1];
#pragma unroll
        for (int q = 0; q < 7; ++q) X.f[5][q] = X.c[q + 1];
        const int64_t off = (int64_t)cur.slot * kBV + lane * 8;
        float r0[8], cin[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) cin[q] = X.c[q];
        if (OP == AT_OP_LAP_UPDATE) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float sum = nbsum(X, q);
                const float six_a = 6.0f * X.c[q];
                const float d = sum - six_a;
                const float tq = p * d;
                r0[q] = X.c[q] + tq;
            }
        } else {
            float bb[8];
            put8(bb, cur.e0, cur.e1);
            const float sixth = 0x1.555556p-3f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float sum = nbsum(X, q);
                const float tq = sum + bb[q];
                r0[q] = tq * sixth;
            }
        }
        apply_tail(g, tail, off, out_ch, in_ch, r0, cin);
        store8(c.out0 + off, r0);
        cur = nxt;
    }
}

// ------------------------------------------------- elementwise (single op)
// Single element-wise struct-for ops, pipelined the same way: the next
// block's inputs are loaded before this block's outputs are stored.
template <int OP>
struct Elem {
    int32_t slot, cell;
    float4 a0, a1, b0, b1, c0, c1, d0, d1;   // up to 4 input rows
};

template <int OP>
__device__ __forceinline__ void fetch_elem(const GridDev &g, const int32_t *__restrict__ recs, const MicroOp &op,
                                           int e, int lane, Elem<OP> &E) {
    const int4 a = reinterpret_cast<const int4 *>(recs + (int64_t)e * kRec)[0];
    E.slot = a.y;
    E.cell = a.x;
    const int64_t off = (int64_t)a.y * kBV + lane * 8;
    auto ld = [&](int ch, float4 &u, float4 &v) {
        const float *p = chan(g, ch) + off;
        u = reinterpret_cast<const float4 *>(p)[0];
        v = reinterpret_cast<const float4 *>(p)[1];
    };
    if (OP == AT_OP_COPY) ld(op.ch[1], E.a0, E.a1);
    if (OP == AT_OP_AXPY) { ld(op.ch[0], E.a0, E.a1); ld(op.ch[1], E.b0, E.b1); }
    if (OP == AT_OP_INC) ld(op.ch[0], E.a0, E.a1);
    if (OP == AT_OP_NORMALISE || OP == AT_OP_MPM_GRID) {
        ld(op.ch[0], E.a0, E.a1);
        ld(op.ch[1], E.b0, E.b1);
        ld(op.ch[1] + 1, E.c0, E.c1);
        ld(op.ch[1] + 2, E.d0, E.d1);
    }
}

__device__ __forceinline__ float4 f4(float a, float b, float c, float d) { return make_float4(a, b, c, d); }

// MLS-MPM grid update of one voxel (I, J, K) of an n^3 domain: velocity from
// momentum where there is mass, gravity along -z (op.p = dt, op.p1 = g), and
// the walls op.p2 nodes thick on every side (AT_OP_MPM_GRID).
__device__ __forceinline__ void mpm_grid_voxel(const MicroOp &op, int n, int I, int J, int K, float m, float mv0,
                                               float mv1, float mv2, float &v0, float &v1, float &v2) {
    v0 = 0.f;
    v1 = 0.f;
    v2 = 0.f;
    if (m > 0.f) {
        v0 = mv0 / m;
        v1 = mv1 / m;
        v2 = mv2 / m;
        v2 = v2 - op.p * op.p1;
        const int bound = (int)op.p2;
        if (I < bound && v0 < 0.f) v0 = 0.f;
        if (I > n - bound && v0 > 0.f) v0 = 0.f;
        if (J < bound && v1 < 0.f) v1 = 0.f;
        if (J > n - bound && v1 > 0.f) v1 = 0.f;
        if (K < bound && v2 < 0.f) v2 = 0.f;
        if (K > n - bound && v2 > 0.f) v2 = 0.f;
    }
}

template <int OP, int KIND, bool CHECK>
__global__ __launch_bounds__(64) void k_elem(GridDev g, const int32_t *__restrict__ recs, MicroOp op) {
    const int lane = threadIdx.x;
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    if (lr.lo >= lr.hi) return;
    Elem<OP> cur, nxt;
    fetch_elem<OP>(g, recs, op, __builtin_amdgcn_readfirstlane(lr.lo), lane, cur);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int en = e + lr.step < lr.hi ? e + lr.step : e;
        fetch_elem<OP>(g, recs, op, __builtin_amdgcn_readfirstlane(en), lane, nxt);
        int32_t wslot = cur.slot;
        if (CHECK) {
            const int32_t cell = recs[(int64_t)e * kRec];
            int32_t a = 0;
            if (lane == 0) a = activate_cell<KIND>(g, cell);
            wslot = __builtin_amdgcn_readfirstlane(a);
        }
        const int64_t off = (int64_t)wslot * kBV + lane * 8;
        auto st = [&](int ch, float4 u, float4 v) {
            float *p = chan(g, ch) + off;
            reinterpret_cast<float4 *>(p)[0] = u;
            reinterpret_cast<float4 *>(p)[1] = v;
        };
        if (OP == AT_OP_COPY) {
            st(op.ch[0], cur.a0, cur.a1);
        } else if (OP == AT_OP_AXPY) {
            const float a = op.p;
            const float4 y0 = cur.a0, y1 = cur.a1, x0 = cur.b0, x1 = cur.b1;
            st(op.ch[0], f4(y0.x + a * x0.x, y0.y + a * x0.y, y0.z + a * x0.z, y0.w + a * x0.w),
               f4(y1.x + a * x1.x, y1.y + a * x1.y, y1.z + a * x1.z, y1.w + a * x1.w));
        } else if (OP == AT_OP_INC) {
            const float a = op.p;
            st(op.ch[0], f4(cur.a0.x + a, cur.a0.y + a, cur.a0.z + a, cur.a0.w + a),
               f4(cur.a1.x + a, cur.a1.y + a, cur.a1.z + a, cur.a1.w + a));
        } else if (OP == AT_OP_FILL) {
            const float4 v = f4(op.p, op.p, op.p, op.p);
            for (int q = 0; q < 7; ++q)
                if (op.ch[q] >= 0 && ((op.keep >> q) & 1u)) st(op.ch[q], v, v);
        } else if (OP == AT_OP_NORMALISE) {
            float m[8], mv[3][8];
            put8(m, cur.a0, cur.a1);
            put8(mv[0], cur.b0, cur.b1);
            put8(mv[1], cur.c0, cur.c1);
            put8(mv[2], cur.d0, cur.d1);
            for (int cc = 0; cc < 3; ++cc) {
                if (!((op.keep >> cc) & 1u)) continue;
                float r[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) r[q] = m[q] > 0.f ? mv[cc][q] / m[q] : 0.f;
                st(op.ch[2] + cc, f4(r[0], r[1], r[2], r[3]), f4(r[4], r[5], r[6], r[7]));
            }
        } else if (OP == AT_OP_MPM_GRID) {
            float m[8], mv[3][8], r[3][8];
            put8(m, cur.a0, cur.a1);
            put8(mv[0], cur.b0, cur.b1);
            put8(mv[1], cur.c0, cur.c1);
            put8(mv[2], cur.d0, cur.d1);
            int bi, bj, bk;
            cell_coords(g, cur.cell, bi, bj, bk);
            const int I[2] = {bi * kBS + (lane >> 3), bj * kBS + (lane & 7)};
#pragma unroll
            for (int q = 0; q < 8; ++q) mpm_grid_voxel(op, g.R * kBS, I[0], I[1], bk * kBS + q, m[q], mv[0][q],
                                                       mv[1][q], mv[2][q], r[0][q], r[1][q], r[2][q]);
            for (int cc = 0; cc < 3; ++cc)
                st(op.ch[2] + cc, f4(r[cc][0], r[cc][1], r[cc][2], r[cc][3]), f4(r[cc][4], r[cc][5], r[cc][6], r[cc][7]));
        }
        cur = nxt;
    }
}

// --------------------------------------------- elementwise / fused programs
// Applies a MicroProg per voxel: each op reads its inputs from memory and
// writes its outputs in program order, so ops fused into one task see each
// other's element-wise results exactly as the unfused sequence would.
// Stencil ops inside a fused program read neighbours straight from memory
// (fusion legality guarantees no op of the program writes a state another
// op reads at an offset).

template <int KIND>
__device__ __forceinline__ float rd_nb(const GridDev &g, const float *base, int32_t slot, const int32_t *nbs,
                                       int li, int lj, int lk, int face) {
    int d = 0;
    int ii = li, jj = lj, kk = lk;
    if (face == 0) { ii = li - 1; d = ii < 0; ii &= 7; }
    else if (face == 1) { ii = li + 1; d = ii > 7; ii &= 7; }
    else if (face == 2) { jj = lj - 1; d = jj < 0; jj &= 7; }
    else if (face == 3) { jj = lj + 1; d = jj > 7; jj &= 7; }
    else if (face == 4) { kk = lk - 1; d = kk < 0; kk &= 7; }
    else { kk = lk + 1; d = kk > 7; kk &= 7; }
    const int32_t s = d ? nbs[face] : slot;
    return s >= 0 ? base[(int64_t)s * kBV + ii * 64 + jj * 8 + kk] : 0.f;
}

// Value of channel `base` at voxel (x, y, z) of an n^3 domain with sparse
// semantics (0 outside the domain or in an inactive block); the wave's own
// block is resolved without a root lookup.
template <int KIND>
__device__ __forceinline__ float sample_voxel(const GridDev &g, const float *base, int64_t own_cell, int32_t own_slot,
                                              int x, int y, int z, int n) {
    if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return 0.f;
    const int64_t c = ((int64_t)(x >> 3) * g.R + (y >> 3)) * g.R + (z >> 3);
    const int32_t s = c == own_cell ? own_slot : slot_of<KIND>(g, c);
    return s >= 0 ? base[(int64_t)s * kBV + (x & 7) * 64 + (y & 7) * 8 + (z & 7)] : 0.f;
}

__device__ __forceinline__ float clamp_coord(float p, int n) {
    return p < -2.f ? -2.f : (p > (float)(n + 1) ? (float)(n + 1) : p);
}

// Trilinear sample of channel `base` at point p (clamped as for the
// advection), fixed corner order, weight (wx * wy) * wz, s = s + w * q.
template <int KIND>
__device__ __forceinline__ float sample_point(const GridDev &g, const float *base, int64_t own_cell, int32_t own_slot,
                                              const float p[3], int n) {
    float w[3][2];
    int b0[3];
    for (int d = 0; d < 3; ++d) {
        const float pd = clamp_coord(p[d], n);
        const float bd = floorf(pd);
        const float f = pd - bd;
        b0[d] = (int)bd;
        w[d][0] = 1.0f - f;
        w[d][1] = f;
    }
    float acc = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                const float wt = (w[0][a] * w[1][b]) * w[2][c];
                acc = acc + wt * sample_voxel<KIND>(g, base, own_cell, own_slot, b0[0] + a, b0[1] + b, b0[2] + c, n);
            }
    return acc;
}

// Back-traced point of voxel I over dt: one Euler step, or (rk3) the
// three-stage Runge-Kutta back-trace with v sampled trilinearly at
// p1 = I - (0.5 dt) v1 and p2 = I - (0.75 dt) v2, then
// p = I - dt (2/9 v1 + 1/3 v2 + 4/9 v3); v1 is v at the voxel (offset off).
template <int KIND>
__device__ __forceinline__ void backtrace_point(const GridDev &g, int v0, int64_t own_cell, int32_t own_slot,
                                                int64_t off, const int I[3], float dt, bool rk3, int n, float p[3]) {
    float v1[3];
    for (int d = 0; d < 3; ++d) v1[d] = chan(g, v0 + d)[off];
    if (!rk3) {
        for (int d = 0; d < 3; ++d) p[d] = (float)I[d] - dt * v1[d];
        return;
    }
    const float h1 = 0.5f * dt, h2 = 0.75f * dt;
    float p1[3], v2[3], p2[3], v3[3];
    for (int d = 0; d < 3; ++d) p1[d] = (float)I[d] - h1 * v1[d];
    for (int d = 0; d < 3; ++d) v2[d] = sample_point<KIND>(g, chan(g, v0 + d), own_cell, own_slot, p1, n);
    for (int d = 0; d < 3; ++d) p2[d] = (float)I[d] - h2 * v2[d];
    for (int d = 0; d < 3; ++d) v3[d] = sample_point<KIND>(g, chan(g, v0 + d), own_cell, own_slot, p2, n);
    const float c1 = (float)(2.0 / 9.0), c2 = (float)(1.0 / 3.0), c3 = (float)(4.0 / 9.0);
    for (int d = 0; d < 3; ++d) {
        float sv = c1 * v1[d];
        sv = sv + c2 * v2[d];
        sv = sv + c3 * v3[d];
        p[d] = (float)I[d] - dt * sv;
    }
}

template <int KIND, bool STENCIL>
__global__ __launch_bounds__(64) void k_micro(GridDev g, MicroProg prog) {
    // one wavefront per block; lane l owns voxels [8l, 8l+8) = row
    // (i, j) = (l >> 3, l & 7), handled as two float4 halves
    const int lane = threadIdx.x;
    const int li = lane >> 3, lj = lane & 7;
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int4 rec0 = reinterpret_cast<const int4 *>(g.list + (int64_t)e * kRec)[0];
        const int32_t cell = rec0.x;
        int32_t slot = rec0.y;
        if (prog.verify && !prog.check && __builtin_amdgcn_readfirstlane(slot_of<KIND>(g, cell)) != slot) {
            if (lane == 0) atomicOr(g.hdr + HDR_ERR, ERR_DEMOTED);   // the listed block is no longer active
            continue;
        }
        int32_t nbs[6] = {-1, -1, -1, -1, -1, -1};
        if (STENCIL) {
            Nbs n;
            int32_t c2, s2;
            if (prog.table) read_record<KIND, true>(g, e, c2, s2, n);
            else n = neighbour_slots<KIND>(g, cell);
            for (int f = 0; f < 6; ++f) nbs[f] = n.s[f];
        }
        if (prog.check) {
            int32_t a = 0;
            if (lane == 0) a = activate_cell<KIND>(g, cell);
            slot = __builtin_amdgcn_readfirstlane(a);
        }
        for (int o = 0; o < prog.nops; ++o) {
            const MicroOp &op = prog.ops[o];
            for (int h = 0; h < 2; ++h) {
                const int64_t off = (int64_t)slot * kBV + lane * 8 + 4 * h;
                const int k0 = 4 * h;
                switch (op.op) {
                case AT_OP_AXPY: {
                    float *y = chan(g, op.ch[0]) + off;
                    const float *x = chan(g, op.ch[1]) + off;
                    float4 yv = *reinterpret_cast<float4 *>(y);
                    const float4 xv = *reinterpret_cast<const float4 *>(x);
                    const float a = op.p;
                    yv.x = yv.x + a * xv.x; yv.y = yv.y + a * xv.y;
                    yv.z = yv.z + a * xv.z; yv.w = yv.w + a * xv.w;
                    *reinterpret_cast<float4 *>(y) = yv;
                    break;
                }
                case AT_OP_COPY:
                    *reinterpret_cast<float4 *>(chan(g, op.ch[0]) + off) =
                        *reinterpret_cast<const float4 *>(chan(g, op.ch[1]) + off);
                    break;
                case AT_OP_FILL:
                    for (int q = 0; q < 7; ++q)
                        if (op.ch[q] >= 0 && ((op.keep >> q) & 1u))
                            *reinterpret_cast<float4 *>(chan(g, op.ch[q]) + off) = make_float4(op.p, op.p, op.p, op.p);
                    break;
                case AT_OP_INC: {
                    float4 *x = reinterpret_cast<float4 *>(chan(g, op.ch[0]) + off);
                    float4 v = *x;
                    v.x = v.x + op.p; v.y = v.y + op.p; v.z = v.z + op.p; v.w = v.w + op.p;
                    *x = v;
                    break;
                }
                case AT_OP_NORMALISE: {
                    const float4 m = *reinterpret_cast<const float4 *>(chan(g, op.ch[0]) + off);
                    const float mm[4] = {m.x, m.y, m.z, m.w};
                    for (int cc = 0; cc < 3; ++cc) {
                        if (!((op.keep >> cc) & 1u)) continue;
                        const float4 mv = *reinterpret_cast<const float4 *>(chan(g, op.ch[1] + cc) + off);
                        const float mvv[4] = {mv.x, mv.y, mv.z, mv.w};
                        float r[4];
                        for (int q = 0; q < 4; ++q) r[q] = mm[q] > 0.f ? mvv[q] / mm[q] : 0.f;
                        *reinterpret_cast<float4 *>(chan(g, op.ch[2] + cc) + off) = make_float4(r[0], r[1], r[2], r[3]);
                    }
                    break;
                }
                case AT_OP_MPM_GRID: {
                    const float4 m = *reinterpret_cast<const float4 *>(chan(g, op.ch[0]) + off);
                    const float4 a = *reinterpret_cast<const float4 *>(chan(g, op.ch[1]) + off);
                    const float4 b = *reinterpret_cast<const float4 *>(chan(g, op.ch[1] + 1) + off);
                    const float4 c = *reinterpret_cast<const float4 *>(chan(g, op.ch[1] + 2) + off);
                    const float mm[4] = {m.x, m.y, m.z, m.w}, m0[4] = {a.x, a.y, a.z, a.w},
                                m1[4] = {b.x, b.y, b.z, b.w}, m2[4] = {c.x, c.y, c.z, c.w};
                    int bi, bj, bk;
                    cell_coords(g, cell, bi, bj, bk);
                    float r[3][4];
                    for (int q = 0; q < 4; ++q)
                        mpm_grid_voxel(op, g.R * kBS, bi * kBS + li, bj * kBS + lj, bk * kBS + k0 + q, mm[q], m0[q],
                                       m1[q], m2[q], r[0][q], r[1][q], r[2][q]);
                    for (int cc = 0; cc < 3; ++cc)
                        *reinterpret_cast<float4 *>(chan(g, op.ch[2] + cc) + off) =
                            make_float4(r[cc][0], r[cc][1], r[cc][2], r[cc][3]);
                    break;
                }
                case AT_OP_ADVECT: {
                    // semi-Lagrangian: q at the back-traced point, trilinear
                    const float *Q = chan(g, op.ch[0]);
                    const int n = g.R * 8;
                    int bi, bj, bk;
                    cell_coords(g, cell, bi, bj, bk);
                    float r[4];
                    for (int q = 0; q < 4; ++q) {
                        const int I[3] = {bi * 8 + li, bj * 8 + lj, bk * 8 + k0 + q};
                        float pt[3];
                        backtrace_point<KIND>(g, op.ch[1], cell, slot, off + q, I, op.p, op.p1 != 0.f, n, pt);
                        r[q] = sample_point<KIND>(g, Q, cell, slot, pt, n);
                    }
                    *reinterpret_cast<float4 *>(chan(g, op.ch[2]) + off) = make_float4(r[0], r[1], r[2], r[3]);
                    break;
                }
                case AT_OP_MACCORMACK: {
                    // fwd + 0.5 (q - bwd), clamped to q's corner range at the back-traced point
                    const float *Q = chan(g, op.ch[0]);
                    const int n = g.R * 8;
                    int bi, bj, bk;
                    cell_coords(g, cell, bi, bj, bk);
                    float r[4];
                    for (int q = 0; q < 4; ++q) {
                        const int I[3] = {bi * 8 + li, bj * 8 + lj, bk * 8 + k0 + q};
                        float pt[3];
                        backtrace_point<KIND>(g, op.ch[1], cell, slot, off + q, I, op.p, op.p1 != 0.f, n, pt);
                        int b0[3];
                        for (int d = 0; d < 3; ++d) b0[d] = (int)floorf(clamp_coord(pt[d], n));
                        float lo = 0.f, hi = 0.f;
                        for (int a = 0; a < 2; ++a)
                            for (int b = 0; b < 2; ++b)
                                for (int c = 0; c < 2; ++c) {
                                    const float x = sample_voxel<KIND>(g, Q, cell, slot, b0[0] + a, b0[1] + b,
                                                                       b0[2] + c, n);
                                    if (a + b + c == 0) {
                                        lo = x;
                                        hi = x;
                                    } else {
                                        lo = x < lo ? x : lo;
                                        hi = x > hi ? x : hi;
                                    }
                                }
                        const float dq = Q[off + q] - chan(g, op.ch[3])[off + q];
                        const float h2 = 0.5f * dq;
                        const float val = chan(g, op.ch[2])[off + q] + h2;
                        r[q] = val < lo ? lo : (val > hi ? hi : val);
                    }
                    *reinterpret_cast<float4 *>(chan(g, op.ch[4]) + off) = make_float4(r[0], r[1], r[2], r[3]);
                    break;
                }
                case AT_OP_LAP_UPDATE:
                case AT_OP_JACOBI:
                case AT_OP_DIFFUSE:
                case AT_OP_DIFFUSE_ADJ: {
                    if (!STENCIL) break;
                    const float *A = chan(g, op.ch[0]);
                    float r0[4], r1[4];
                    for (int q = 0; q < 4; ++q) {
                        const int lk = k0 + q;
                        const float a = A[off + q];
                        float nb[6];
                        for (int fc = 0; fc < 6; ++fc) nb[fc] = rd_nb<KIND>(g, A, slot, nbs, li, lj, lk, fc);
                        if (op.op == AT_OP_LAP_UPDATE || op.op == AT_OP_JACOBI) {
                            float s = nb[0] + nb[1];
                            s = s + nb[2]; s = s + nb[3]; s = s + nb[4]; s = s + nb[5];
                            if (op.op == AT_OP_LAP_UPDATE) {
                                const float six_a = 6.0f * a;
                                const float d = s - six_a;
                                const float tq = op.p * d;
                                r0[q] = a + tq;
                            } else {
                                const float tq = s + chan(g, op.ch[1])[off + q];
                                r0[q] = tq * 0x1.555556p-3f;
                            }
                        } else {
                            const float *K = chan(g, op.ch[1]);
                            const float kc = K[off + q];
                            if (op.op == AT_OP_DIFFUSE) {
                                float f = 0.f;
                                for (int fc = 0; fc < 6; ++fc) {
                                    const float kf = 0.5f * (kc + rd_nb<KIND>(g, K, slot, nbs, li, lj, lk, fc));
                                    f = f + kf * (nb[fc] - a);
                                }
                                r0[q] = a + op.p * f;
                            } else {
                                const float *Ln = chan(g, op.ch[2]);
                                const float l = Ln[off + q];
                                float f = 0.f, q2 = 0.f;
                                for (int fc = 0; fc < 6; ++fc) {
                                    const float ln = rd_nb<KIND>(g, Ln, slot, nbs, li, lj, lk, fc);
                                    const float kf = 0.5f * (kc + rd_nb<KIND>(g, K, slot, nbs, li, lj, lk, fc));
                                    f = f + kf * (ln - l);
                                    q2 = q2 + (nb[fc] - a) * (l - ln);
                                }
                                r0[q] = l + op.p * f;
                                r1[q] = chan(g, op.ch[4])[off + q] + (op.p * 0.5f) * q2;
                            }
                        }
                    }
                    const int outc = op.op == AT_OP_LAP_UPDATE ? op.ch[1]
                                   : op.op == AT_OP_JACOBI ? op.ch[2]
                                   : op.op == AT_OP_DIFFUSE ? op.ch[2] : op.ch[3];
                    *reinterpret_cast<float4 *>(chan(g, outc) + off) = make_float4(r0[0], r0[1], r0[2], r0[3]);
                    if (op.op == AT_OP_DIFFUSE_ADJ)
                        *reinterpret_cast<float4 *>(chan(g, op.ch[4]) + off) = make_float4(r1[0], r1[1], r1[2], r1[3]);
                    break;
                }
                default:
                    break;
                }
            }
        }
    }
}

// ------------------------------------------- advection over staged tiles
// A fused (or single) struct-for whose ops sample channels at back-traced
// points (ADVECT, MACCORMACK), possibly with element-wise ops: one
// workgroup of 512 threads per listed block stages, in LDS, the block plus a
// 2-voxel halo (12^3 voxels; this workload's back-traces reach 1.34 voxels)
// of every channel the node samples and, for RK3 back-traces, of the three
// velocity channels -- coalesced rows, one root lookup per neighbour block
// for the whole tile -- and then runs the ops per voxel in program order.
// A trilinear sample whose 8 corners lie in the tile reads LDS, in the same
// corner order and arithmetic as sample_point, so results are bit-identical
// to the per-voxel interpreter; a point outside the tile reads the grid as
// before.  Fusion legality guarantees that no op of the node writes a
// channel another op samples, so the staged tiles stay valid for the whole
// node.
constexpr int kTC = 4;                            // tile voxels a thread loads before storing them

// Tile position of a point coordinate's lower corner: the corner pair
// (b0, b0 + 1) lies in the tile when 0 <= b0 - origin <= kTE - 2.
__device__ __forceinline__ float tile_sample(const float *T, const int lb[3], const float w[3][2]) {
    float acc = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                const float wt = (w[0][a] * w[1][b]) * w[2][c];
                acc = acc + wt * T[((lb[0] + a) * kTE + (lb[1] + b)) * kTE + (lb[2] + c)];
            }
    return acc;
}

// The rare sample outside the staged tile, inline but one corner at a time
// (no unrolling, so it adds few registers to the staged path): the
// arithmetic of sample_point, corner for corner.
template <int KIND>
__device__ __forceinline__ float sample_far(const GridDev &g, const float *base, int64_t cell, int32_t slot,
                                            const float p[3], int n) {
    float w0[3], w1[3];
    int b0[3];
    for (int d = 0; d < 3; ++d) {
        const float pd = clamp_coord(p[d], n);
        const float bd = floorf(pd);
        const float f = pd - bd;
        b0[d] = (int)bd;
        w0[d] = 1.0f - f;
        w1[d] = f;
    }
    float acc = 0.f;
#pragma nounroll
    for (int q = 0; q < 8; ++q) {
        const int a = q >> 2, b = (q >> 1) & 1, c = q & 1;
        const float wt = ((a ? w1[0] : w0[0]) * (b ? w1[1] : w0[1])) * (c ? w1[2] : w0[2]);
        acc = acc + wt * sample_voxel<KIND>(g, base, cell, slot, b0[0] + a, b0[1] + b, b0[2] + c, n);
    }
    return acc;
}

// Range (lo, hi) of the 8 corners from (b0, b1, b2), outside the tile.
template <int KIND>
__device__ __forceinline__ void corners_far(const GridDev &g, const float *Q, int64_t cell, int32_t slot, int b0,
                                            int b1, int b2, int n, float &lo, float &hi) {
#pragma nounroll
    for (int q = 0; q < 8; ++q) {
        const float x = sample_voxel<KIND>(g, Q, cell, slot, b0 + (q >> 2), b1 + ((q >> 1) & 1), b2 + (q & 1), n);
        if (q == 0) {
            lo = x;
            hi = x;
        } else {
            lo = x < lo ? x : lo;
            hi = x > hi ? x : hi;
        }
    }
}

// Trilinear sample of channel ch at p: from the staged tile T (origin o,
// the block's first voxel minus 2) when all corners lie in it, else from the
// grid (sample_point).  Same clamp, weights, corner order and arithmetic.
template <int KIND>
__device__ __forceinline__ float sample_staged(const GridDev &g, const float *T, const int o[3], const float *base,
                                               int64_t cell, int32_t slot, const float p[3], int n) {
    float w[3][2];
    int lb[3];
    bool in = T != nullptr;
    for (int d = 0; d < 3; ++d) {
        const float pd = clamp_coord(p[d], n);
        const float bd = floorf(pd);
        const float f = pd - bd;
        lb[d] = (int)bd - o[d];
        in = in && lb[d] >= 0 && lb[d] <= kTE - 2;
        w[d][0] = 1.0f - f;
        w[d][1] = f;
    }
    if (in) return tile_sample(T, lb, w);
    return sample_far<KIND>(g, base, cell, slot, p, n);
}

template <int KIND>
__device__ __forceinline__ const float *staged(const TileProg &tp, const float *tiles, int ch) {
    for (int q = 0; q < tp.nt; ++q)
        if (tp.tch[q] == ch) return tiles + q * kT3;
    return nullptr;
}

// The sampling state of a back-traced point p shared by every field sampled
// there: the 8 corner weights (w0 * w1) * w2 in corner order, and the tile
// index of the lower corner, or -1 when a corner lies outside the tile.
// Same clamp, floor and products as sample_staged.
__device__ __forceinline__ int trace_tile(const float p[3], const int o[3], int n, float wt[8]) {
    float w[3][2];
    int lb[3];
    bool in = true;
    for (int d = 0; d < 3; ++d) {
        const float pd = clamp_coord(p[d], n);
        const float bd = floorf(pd);
        const float f = pd - bd;
        lb[d] = (int)bd - o[d];
        in = in && lb[d] >= 0 && lb[d] <= kTE - 2;
        w[d][0] = 1.0f - f;
        w[d][1] = f;
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) wt[(a * 2 + b) * 2 + c] = (w[0][a] * w[1][b]) * w[2][c];
    return in ? (lb[0] * kTE + lb[1]) * kTE + lb[2] : -1;
}

// tile_sample with the weights of trace_tile; T points at the lower corner.
__device__ __forceinline__ float tile_sum(const float *T, const float wt[8]) {
    float acc = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) acc = acc + wt[(a * 2 + b) * 2 + c] * T[(a * kTE + b) * kTE + c];
    return acc;
}

// LDS layout (dynamic): the nt sampled tiles, then the velocity: three
// tiles when staged for RK3 back-traces, else the block's own 512 voxels of
// each component when every sampling op shares one velocity (v0 >= 0).
__host__ __device__ inline int tile_lds_floats(const TileProg &tp) {
    return tp.nt * kT3 + (tp.vstage ? 3 * kT3 : (tp.v0 >= 0 ? 3 * kBV : 0));
}

// Tile voxel number e (0 .. kT3 - 1) in source order: the block's own 512
// voxels, then the 2-voxel face slabs of the neighbours across i-, i+, j-,
// j+, k-, k+ (128 each), the twelve edge pieces (32 each: i and j sides,
// then i and k, then j and k) and the eight corners (8 each), every piece in
// its source block's memory order (k fastest).  Consecutive numbers are
// then consecutive addresses along the pieces' rows, so a wave's staging
// load touches few cache lines.  Returns the neighbour (0 .. 26, as s_nb)
// and sets the voxel's offset in that block and its tile position.
__device__ __forceinline__ int tile_src(int e, int &src, int &tpos) {
    int d0 = 0, d1 = 0, d2 = 0, l;
    if (e < 512) {
        l = e;
    } else if (e < 1280) {
        const int f = (e - 512) >> 7, sg = (f & 1) ? 1 : -1;
        l = (e - 512) & 127;
        d0 = f >> 1 == 0 ? sg : 0;
        d1 = f >> 1 == 1 ? sg : 0;
        d2 = f >> 1 == 2 ? sg : 0;
    } else if (e < 1664) {
        const int m = (e - 1280) >> 5, pr = m >> 2;
        const int sa = (m & 2) ? 1 : -1, sb = (m & 1) ? 1 : -1;
        l = (e - 1280) & 31;
        d0 = pr <= 1 ? sa : 0;
        d1 = pr == 0 ? sb : (pr == 2 ? sa : 0);
        d2 = pr >= 1 ? sb : 0;
    } else {
        const int c = (e - 1664) >> 3;
        l = (e - 1664) & 7;
        d0 = (c & 4) ? 1 : -1;
        d1 = (c & 2) ? 1 : -1;
        d2 = (c & 1) ? 1 : -1;
    }
    const int bk = d2 ? 1 : 3, bj = d1 ? 1 : 3;              // log2 of the piece's extent
    const int sk = l & ((1 << bk) - 1), sj = (l >> bk) & ((1 << bj) - 1), si = l >> (bk + bj);
    const int i = d0 < 0 ? 6 + si : si, j = d1 < 0 ? 6 + sj : sj, k = d2 < 0 ? 6 + sk : sk;
    src = i * 64 + j * 8 + k;
    const int ti = d0 < 0 ? si : (d0 ? 10 + si : 2 + si), tj = d1 < 0 ? sj : (d1 ? 10 + sj : 2 + sj),
              tk = d2 < 0 ? sk : (d2 ? 10 + sk : 2 + sk);
    tpos = (ti * kTE + tj) * kTE + tk;
    return (d0 + 1) * 9 + (d1 + 1) * 3 + (d2 + 1);
}

// Six waves per SIMD (3 workgroups per CU instead of the 2 its 93 VGPRs
// allow): a few spilled values, 15% faster on the advection workloads.
template <int KIND, int NT, bool VS>
__global__ __launch_bounds__(kTT) __attribute__((amdgpu_waves_per_eu(6))) void k_tile_micro(GridDev g, TileProg tp) {
    extern __shared__ float s_t[];
    __shared__ int32_t s_nb[27];
    const int tid = threadIdx.x;
    const int n = g.R * kBS;
    float *vs = s_t + tp.nt * kT3;                       // velocity: tiles or the block's voxels
    const float *vt = tp.vstage ? vs : nullptr;
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int4 rec0 = reinterpret_cast<const int4 *>(g.list + (int64_t)e * kRec)[0];
        const int32_t cell = rec0.x, slot = rec0.y;
        int bi, bj, bk;
        cell_coords(g, cell, bi, bj, bk);
        if (tid < 27) {
            const int ni = bi + tid / 9 - 1, nj = bj + (tid / 3) % 3 - 1, nk = bk + tid % 3 - 1;
            int32_t sl = -1;
            if (ni >= 0 && nj >= 0 && nk >= 0 && ni < g.R && nj < g.R && nk < g.R)
                sl = tid == 13 ? slot : slot_of<KIND>(g, ((int64_t)ni * g.R + nj) * g.R + nk);
            s_nb[tid] = sl;
        }
        __syncthreads();
        // every load of the tile first (a valid dummy address where the block
        // is outside the domain or inactive, zeroed by a select), then the
        // LDS stores, so the loads overlap instead of each waiting for the
        // store after it; voxels in source order (tile_src)
        // (in chunks of kTC voxels per thread, which bounds the registers)
        constexpr int NIT = (kT3 + kTT - 1) / kTT, NC = NT + (VS ? 3 : 0);
#pragma unroll
        for (int c0 = 0; c0 < NIT; c0 += kTC) {
            float val[kTC][NC];
            bool ok[kTC];
            int tpos[kTC];
#pragma unroll
            for (int u = 0; u < kTC; ++u) {
                const int it = c0 + u;
                if (it >= NIT) break;
                const int t = tid + it * kTT < kT3 ? tid + it * kTT : 0;
                int src;
                const int32_t sl = s_nb[tile_src(t, src, tpos[u])];   // -1 outside the domain or inactive
                ok[u] = sl >= 0;
                const int64_t o = (int64_t)(sl >= 0 ? sl : slot) * kBV + src;
#pragma unroll
                for (int q = 0; q < NT; ++q) val[u][q] = chan(g, tp.tch[q])[o];
#pragma unroll
                for (int d = 0; d < (VS ? 3 : 0); ++d) val[u][NT + d] = chan(g, tp.v0 + d)[o];
            }
#pragma unroll
            for (int u = 0; u < kTC; ++u) {
                const int it = c0 + u;
                if (it >= NIT) break;
                if (tid + it * kTT < kT3) {
                    const int t = tpos[u];
#pragma unroll
                    for (int q = 0; q < NT; ++q) s_t[q * kT3 + t] = ok[u] ? val[u][q] : 0.f;
#pragma unroll
                    for (int d = 0; d < (VS ? 3 : 0); ++d) vs[d * kT3 + t] = ok[u] ? val[u][NT + d] : 0.f;
                }
            }
            __builtin_amdgcn_sched_barrier(0);   // the next chunk's loads after these stores
        }
        if (!VS && tp.v0 >= 0)
            for (int vx = tid; vx < kBV; vx += kTT)
#pragma unroll
                for (int d = 0; d < 3; ++d) vs[d * kBV + vx] = chan(g, tp.v0 + d)[(int64_t)slot * kBV + vx];
        __syncthreads();
        const int org[3] = {bi * kBS - 2, bj * kBS - 2, bk * kBS - 2};
#pragma nounroll
        for (int vx = tid; vx < kBV; vx += kTT) {
            const int li = vx >> 6, lj = (vx >> 3) & 7, lk = vx & 7;
            const int I[3] = {bi * kBS + li, bj * kBS + lj, bk * kBS + lk};
            const int64_t off = (int64_t)slot * kBV + vx;
            // the back-traced point of the last (velocity, dt, rk3) used
            float pt[3] = {0.f, 0.f, 0.f}, pdt = 0.f, prk = -1.f;
            int pv = -1;
            // its sampling state (trace_tile), shared by the fields sampled there
            float wt[8];
            int lbase = -1;
            for (int oi = 0; oi < tp.prog.nops; ++oi) {
                const MicroOp &op = tp.prog.ops[oi];
                if (op.op == AT_OP_ADVECT || op.op == AT_OP_MACCORMACK) {
                    if (!(op.ch[1] == pv && op.p == pdt && op.p1 == prk)) {
                        float v1[3];
                        if (op.ch[1] == tp.v0 && tp.vstage) {
                            const int c = ((li + 2) * kTE + (lj + 2)) * kTE + (lk + 2);
                            for (int d = 0; d < 3; ++d) v1[d] = vs[d * kT3 + c];
                        } else if (op.ch[1] == tp.v0) {
                            for (int d = 0; d < 3; ++d) v1[d] = vs[d * kBV + vx];
                        } else {
                            for (int d = 0; d < 3; ++d) v1[d] = chan(g, op.ch[1] + d)[off];
                        }
                        if (!VS || op.p1 == 0.f) {   // (every RK3 op stages velocity tiles)
                            for (int d = 0; d < 3; ++d) pt[d] = (float)I[d] - op.p * v1[d];
                        } else {
                            const float *vtile = op.ch[1] == tp.v0 ? vt : nullptr;
                            const float h1 = 0.5f * op.p, h2 = 0.75f * op.p;
                            float p1[3], v2[3], p2[3], v3[3];
                            for (int d = 0; d < 3; ++d) p1[d] = (float)I[d] - h1 * v1[d];
                            for (int d = 0; d < 3; ++d)
                                v2[d] = sample_staged<KIND>(g, vtile ? vtile + d * kT3 : nullptr, org,
                                                            chan(g, op.ch[1] + d), cell, slot, p1, n);
                            for (int d = 0; d < 3; ++d) p2[d] = (float)I[d] - h2 * v2[d];
                            for (int d = 0; d < 3; ++d)
                                v3[d] = sample_staged<KIND>(g, vtile ? vtile + d * kT3 : nullptr, org,
                                                            chan(g, op.ch[1] + d), cell, slot, p2, n);
                            const float c1 = (float)(2.0 / 9.0), c2 = (float)(1.0 / 3.0), c3 = (float)(4.0 / 9.0);
                            for (int d = 0; d < 3; ++d) {
                                float sv = c1 * v1[d];
                                sv = sv + c2 * v2[d];
                                sv = sv + c3 * v3[d];
                                pt[d] = (float)I[d] - op.p * sv;
                            }
                        }
                        pdt = op.p;
                        prk = op.p1;
                        pv = op.ch[1];
                        lbase = trace_tile(pt, org, n, wt);
                    }
                    const float *Q = chan(g, op.ch[0]);
                    const float *qt = staged<KIND>(tp, s_t, op.ch[0]);
                    const bool in = qt != nullptr && lbase >= 0;
                    if (op.op == AT_OP_ADVECT) {
                        chan(g, op.ch[2])[off] =
                            in ? tile_sum(qt + lbase, wt) : sample_far<KIND>(g, Q, cell, slot, pt, n);
                    } else {
                        float lo = 0.f, hi = 0.f;
                        if (in) {
                            const float *T = qt + lbase;
                            for (int a = 0; a < 2; ++a)
                                for (int b = 0; b < 2; ++b)
                                    for (int c = 0; c < 2; ++c) {
                                        const float x = T[(a * kTE + b) * kTE + c];
                                        if (a + b + c == 0) {
                                            lo = x;
                                            hi = x;
                                        } else {
                                            lo = x < lo ? x : lo;
                                            hi = x > hi ? x : hi;
                                        }
                                    }
                        } else {
                            int b0[3];
                            for (int d = 0; d < 3; ++d) b0[d] = (int)floorf(clamp_coord(pt[d], n));
                            corners_far<KIND>(g, Q, cell, slot, b0[0], b0[1], b0[2], n, lo, hi);
                        }
                        const float dq = Q[off] - chan(g, op.ch[3])[off];
                        const float h2 = 0.5f * dq;
                        const float val = chan(g, op.ch[2])[off] + h2;
                        chan(g, op.ch[4])[off] = val < lo ? lo : (val > hi ? hi : val);
                    }
                } else if (op.op == AT_OP_COPY) {
                    chan(g, op.ch[0])[off] = chan(g, op.ch[1])[off];
                } else if (op.op == AT_OP_AXPY) {
                    float *y = chan(g, op.ch[0]) + off;
                    *y = *y + op.p * chan(g, op.ch[1])[off];
                } else if (op.op == AT_OP_INC) {
                    float *x = chan(g, op.ch[0]) + off;
                    *x = *x + op.p;
                } else if (op.op == AT_OP_FILL) {
                    for (int q = 0; q < 7; ++q)
                        if (op.ch[q] >= 0 && ((op.keep >> q) & 1u)) chan(g, op.ch[q])[off] = op.p;
                }
            }
        }
        __syncthreads();   // the next block restages the tiles
    }
}

// ---------------------------------------------------- two-level transfers
// A coarse grid has half the fine domain edge, so fine block (bi, bj, bk)
// lies under coarse block (bi/2, bj/2, bk/2), in its octant
// (bi&1, bj&1, bk&1) of 4^3 voxels.  One wavefront per listed fine block.

// Restriction y[I/2] += w * x[I].  Lane l owns coarse voxel (l>>4, (l>>2)&3,
// l&3) of the octant and adds its 8 children (two float2 loads per child
// row pair) one at a time, in ascending order of their index in the fine
// block.  The fine blocks under one coarse block write disjoint octants and a
// fine block is listed once, so the read-modify-write needs no atomics; the
// coarse block is activated by lane 0 first (CHECK) or looked up.
template <int KF, int KC, bool CHECK>
__global__ __launch_bounds__(64) void k_restrict(GridDev f, GridDev c, const float *__restrict__ x, float *y,
                                                 float w, int verify) {
    const int lane = threadIdx.x;
    const ListRange lr = list_range(f.hdr[HDR_COUNT]);
    const int ci = lane >> 4, cj = (lane >> 2) & 3, ck = lane & 3;
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int4 r = reinterpret_cast<const int4 *>(f.list + (int64_t)e * kRec)[0];
        int bi, bj, bk;
        cell_coords(f, r.x, bi, bj, bk);
        const int64_t cc = ((int64_t)(bi >> 1) * c.R + (bj >> 1)) * c.R + (bk >> 1);
        int32_t cs;
        if (CHECK) {
            int32_t a = 0;
            if (lane == 0) a = activate_cell<KC>(c, cc);
            cs = __builtin_amdgcn_readfirstlane(a);
        } else {
            cs = __builtin_amdgcn_readfirstlane(slot_of<KC>(c, cc));
            // a demoted check whose block is not active: an optimizer error
            if (verify && cs < 0 && lane == 0) atomicOr(c.hdr + HDR_ERR, ERR_DEMOTED);
        }
        if (cs < 0) continue;
        const float *xp = x + (int64_t)r.y * kBV + (2 * ci) * 64 + (2 * cj) * 8 + 2 * ck;
        float *yp = y + (int64_t)cs * kBV + ((bi & 1) * 4 + ci) * 64 + ((bj & 1) * 4 + cj) * 8 + (bk & 1) * 4 + ck;
        float2 ch[4];
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) ch[ab] = *reinterpret_cast<const float2 *>(xp + (ab >> 1) * 64 + (ab & 1) * 8);
        float acc = *yp;
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) {
            const float t0 = w * ch[ab].x;
            acc = acc + t0;
            const float t1 = w * ch[ab].y;
            acc = acc + t1;
        }
        *yp = acc;
    }
}

// Prolongation by injection x[I] += y[I/2].  Lane l owns fine row
// (l>>3, l&7, 0..7), which reads 4 consecutive coarse voxels (one float4);
// an inactive coarse block reads as zeros.
template <int KF, int KC, bool CHECK>
__global__ __launch_bounds__(64) void k_prolong(GridDev f, GridDev c, const float *__restrict__ y, float *x,
                                                int verify) {
    const int lane = threadIdx.x;
    const ListRange lr = list_range(f.hdr[HDR_COUNT]);
    const int li = lane >> 3, lj = lane & 7;
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int4 r = reinterpret_cast<const int4 *>(f.list + (int64_t)e * kRec)[0];
        int bi, bj, bk;
        cell_coords(f, r.x, bi, bj, bk);
        const int64_t cc = ((int64_t)(bi >> 1) * c.R + (bj >> 1)) * c.R + (bk >> 1);
        const int32_t cs = __builtin_amdgcn_readfirstlane(slot_of<KC>(c, cc));
        int32_t fs = r.y;
        if (CHECK) {
            int32_t a = 0;
            if (lane == 0) a = activate_cell<KF>(f, r.x);
            fs = __builtin_amdgcn_readfirstlane(a);
            if (fs < 0) continue;
        } else if (verify && __builtin_amdgcn_readfirstlane(slot_of<KF>(f, r.x)) != fs) {
            if (lane == 0) atomicOr(f.hdr + HDR_ERR, ERR_DEMOTED);   // the listed block is no longer active
            continue;
        }
        float4 yv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (cs >= 0)
            yv = *reinterpret_cast<const float4 *>(y + (int64_t)cs * kBV + ((bi & 1) * 4 + (li >> 1)) * 64 +
                                                   ((bj & 1) * 4 + (lj >> 1)) * 8 + (bk & 1) * 4);
        float *xp = x + (int64_t)fs * kBV + lane * 8;
        const float4 a = reinterpret_cast<const float4 *>(xp)[0];
        const float4 b = reinterpret_cast<const float4 *>(xp)[1];
        reinterpret_cast<float4 *>(xp)[0] = make_float4(a.x + yv.x, a.y + yv.x, a.z + yv.y, a.w + yv.y);
        reinterpret_cast<float4 *>(xp)[1] = make_float4(b.x + yv.z, b.y + yv.z, b.z + yv.w, b.w + yv.w);
    }
}

// ------------------------------------------------------------ batched Jacobi
// Many independent pointer-rooted grids of one domain size share a leaf
// pool.  The device work list holds (grid, root cell) pairs as
// grid * R^3 + cell; grid g is active in global iteration i when
// window[g].start <= i < window[g].end, with i = clock + it, so one captured
// sequence of launches serves any mix of grids admitted at different times.
// One wavefront per listed block, the same arithmetic (and operation order)
// as the single-grid Jacobi and copy kernels; the block's slot and its
// neighbours' come from a record per work entry, so the sweep does no root
// lookups.

// Records of the work list, rebuilt at the start of every call from the
// roots as they are then: {slot, grid, nb0, nb1}, {nb2, nb3, nb4, nb5}.
__global__ __launch_bounds__(256) void k_batch_records(BatchDev d) {
    const int n = *d.count;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int32_t w = d.work[e];
        if (w < 0) {                       // an entry without a block (see k_batch_admit)
            d.rec[2 * e] = make_int4(-1, 0, -1, -1);
            d.rec[2 * e + 1] = make_int4(-1, -1, -1, -1);
            continue;
        }
        const int gid = w / d.ncells;
        const int32_t cell = w - gid * d.ncells;
        const int32_t *root = d.roots + (int64_t)gid * d.ncells;
        const int bi = cell / d.R2, r = cell - bi * d.R2, bj = r / d.R, bk = r - bj * d.R;
        auto nb = [&](bool ok, int32_t c) {
            const int32_t s = ok ? root[c] : -1;
            return s >= 0 ? s : -1;
        };
        d.rec[2 * e] = make_int4(root[cell], gid, nb(bi > 0, cell - d.R2), nb(bi < d.R - 1, cell + d.R2));
        d.rec[2 * e + 1] = make_int4(nb(bj > 0, cell - d.R), nb(bj < d.R - 1, cell + d.R), nb(bk > 0, cell - 1),
                                     nb(bk < d.R - 1, cell + 1));
    }
}

// Range of work entries a wavefront walks when a workgroup holds W
// wavefronts: the workgroup's XCD slice as in list_range, each wavefront a
// virtual workgroup of its own.
template <int W>
__device__ __forceinline__ ListRange wave_range(int count) {
    const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
    const int x = blockIdx.x % nx;
    const int local = (blockIdx.x / nx) * W + (int)(threadIdx.x >> 6);
    const int per = (gridDim.x / nx) * W;
    const int lo = (int)(((int64_t)count * x) / nx);
    const int hi = (int)(((int64_t)count * (x + 1)) / nx);
    return {lo + local, hi, per};
}

template <bool COPY, int W>
__global__ __launch_bounds__(64 * W) void k_batch(BatchDev d, int it) {
    const int lane = threadIdx.x & 63;
    const int64_t now = *d.clock + it;
    const ListRange lr = wave_range<W>(*d.count);
    const int4 *__restrict__ rec = d.rec;
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int4 r0 = rec[2 * e];
        const int gid = r0.y;
        if (now < d.window[2 * gid] || now >= d.window[2 * gid + 1]) continue;
        const int32_t slot = r0.x;
        if (slot < 0) continue;
        const int64_t off = (int64_t)slot * kBV + lane * 8;
        if (COPY) {
            const float4 a = reinterpret_cast<const float4 *>(d.xn + off)[0];
            const float4 b = reinterpret_cast<const float4 *>(d.xn + off)[1];
            reinterpret_cast<float4 *>(d.x + off)[0] = a;
            reinterpret_cast<float4 *>(d.x + off)[1] = b;
            continue;
        }
        const int4 r1 = rec[2 * e + 1];
        Nbs n;
        n.s[0] = r0.z; n.s[1] = r0.w; n.s[2] = r1.x; n.s[3] = r1.y; n.s[4] = r1.z; n.s[5] = r1.w;
        Row X;
        load_row(d.x, slot, n, lane, X);
        float b[8], r[8];
        put8(b, reinterpret_cast<const float4 *>(d.b + off)[0], reinterpret_cast<const float4 *>(d.b + off)[1]);
        const float sixth = 0x1.555556p-3f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float sum = nbsum(X, q);
            const float tq = sum + b[q];
            r[q] = tq * sixth;
        }
        store8(d.xn + off, r);
    }
}

// The batched Jacobi sweep in the form of k_stencil_lds: each wavefront
// keeps its own LDS rows and faces, loads the next entry's block while it
// computes this one (records, window and slots included), and stages the
// block's rows and lateral faces through LDS.  Same arithmetic and order as
// k_batch, so the same results bit for bit.
template <int W>
__global__ __launch_bounds__(64 * W) void k_batch_lds(BatchDev d, int it) {
    __shared__ float4 s_own_w[W][2][64];
    __shared__ float4 s_face_w[W][2][4][8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float4 (*s_own)[64] = s_own_w[wv];
    float4 (*s_face)[4][8] = s_face_w[wv];
    const int li = lane >> 3, lj = lane & 7;
    const int f = lane >> 4, frow = (lane & 15) >> 1, fh = lane & 1;
    const float4 *src[4] = {li > 0 ? &s_own[0][lane - 8] : &s_face[0][0][lj],
                            li < 7 ? &s_own[0][lane + 8] : &s_face[0][1][lj],
                            lj > 0 ? &s_own[0][lane - 1] : &s_face[0][2][li],
                            lj < 7 ? &s_own[0][lane + 1] : &s_face[0][3][li]};
    const int hstride[4] = {li > 0 ? 64 : 32, li < 7 ? 64 : 32, lj > 0 ? 64 : 32, lj < 7 ? 64 : 32};
    const int64_t now = *d.clock + it;
    const ListRange lr = wave_range<W>(*d.count);
    if (lr.lo >= lr.hi) return;
    StencilCh c{};
    c.tin[0] = d.x;
    c.ein = d.b;
    c.out0 = d.xn;
    // entry e's block (a dummy valid slot when it has none), and whether its
    // grid sweeps at this iteration
    auto fetch = [&](int e, BlkL<true> &B) {
        const int4 r0 = d.rec[2 * e], r1 = d.rec[2 * e + 1];
        const int gid = r0.y;
        bool on = r0.x >= 0 && gid >= 0 && gid < d.max_grids;
        if (on) on = now >= d.window[2 * gid] && now < d.window[2 * gid + 1];
        fetch_rec_lds<true>(c, make_int4(0, r0.x >= 0 ? r0.x : 0, r0.z, r0.w), r1, lane, B);
        return on;
    };
    BlkL<true> cur, nxt;
    bool on_cur = fetch(__builtin_amdgcn_readfirstlane(lr.lo), cur);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int en = e + lr.step < lr.hi ? e + lr.step : e;
        const bool on_nxt = fetch(__builtin_amdgcn_readfirstlane(en), nxt);
        if (on_cur) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // the last block's reads come first
            s_own[0][lane] = cur.c0;
            s_own[1][lane] = cur.c1;
            s_face[fh][f][frow] = cur.face;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // then this block's writes
            Row X;
            put8(X.c, cur.c0, cur.c1);
#pragma unroll
            for (int q = 0; q < 4; ++q) put8(X.f[q], src[q][0], src[q][hstride[q]]);
            X.f[4][0] = cur.km;
            X.f[5][7] = cur.kp;
#pragma unroll
            for (int q = 1; q < 8; ++q) X.f[4][q] = X.c[q - 1];
#pragma unroll
            for (int q = 0; q < 7; ++q) X.f[5][q] = X.c[q + 1];
            float bb[8], r0[8];
            put8(bb, cur.e0, cur.e1);
            const float sixth = 0x1.555556p-3f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float sum = nbsum(X, q);
                const float tq = sum + bb[q];
                r0[q] = tq * sixth;
            }
            store8(d.xn + (int64_t)cur.slot * kBV + lane * 8, r0);
        }
        cur = nxt;
        on_cur = on_nxt;
    }
}

__global__ void k_batch_tick(BatchDev d, int iters) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *d.clock += iters;
}

// Batch updates.  The pool's free slots are a stack in device memory whose
// height only the host tracks, so the slots an admission takes and a
// retirement returns never cross to the host.  One workgroup of 128 threads
// per pool block (a float4 each); the descriptors come as kernel arguments.
__global__ __launch_bounds__(256) void k_batch_init(BatchDev d) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.pool; i += gridDim.x * blockDim.x)
        d.free_slots[i] = i;
}

// Retirement: x of the grid's blocks out (when asked), its slots back on the
// stack, its root cells and window cleared.
__global__ __launch_bounds__(128) void k_batch_retire(BatchDev d, BatchRetireArgs a) {
    const int w = blockIdx.x, t = threadIdx.x;
    int k = 0;
    while (k + 1 < a.n && w >= a.it[k + 1].first) ++k;
    const BatchRetireItem &it = a.it[k];
    const int i = w - it.first;
    const int32_t s = it.slots[i];
    if (it.x_out && s >= 0 && s < d.pool)
        reinterpret_cast<float4 *>(it.x_out + (int64_t)i * kBV)[t] =
            reinterpret_cast<const float4 *>(d.x + (int64_t)s * kBV)[t];
    if (t == 0) {
        d.free_slots[it.q + i] = s;
        const int32_t c = it.cells[i];
        if (c >= 0 && c < d.ncells) d.roots[(int64_t)it.gid * d.ncells + c] = -1;
        if (i == 0) {
            d.window[2 * it.gid] = 0;
            d.window[2 * it.gid + 1] = 0;
        }
    }
}

// Admission (the first adm_blocks workgroups): a slot off the stack per
// block, b copied in, x and xn zeroed, the root cell pointed at the slot,
// and the window [clock, clock + iters) read from the device clock, i.e. in
// stream order after every sweep enqueued before.  The other workgroups, one
// per resident grid, write the work list: entries grid * R^3 + cell in the
// order given (a cell outside the root gives an entry without a block).
__global__ __launch_bounds__(128) void k_batch_admit(BatchDev d, BatchAdmitArgs a) {
    const int w = blockIdx.x, t = threadIdx.x;
    if (w == 0 && t == 0) *d.count = a.count;
    if (w < a.adm_blocks) {
        int k = 0;
        while (k + 1 < a.nadm && w >= a.it[k + 1].first) ++k;
        const BatchAdmitItem &it = a.it[k];
        const int i = w - it.first;
        const int32_t s = d.free_slots[it.p + i];
        const int64_t o = (int64_t)s * kBV;
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        reinterpret_cast<float4 *>(d.b + o)[t] = reinterpret_cast<const float4 *>(it.b + (int64_t)i * kBV)[t];
        reinterpret_cast<float4 *>(d.x + o)[t] = z;
        reinterpret_cast<float4 *>(d.xn + o)[t] = z;
        if (t == 0) {
            it.slots[i] = s;
            const int32_t c = it.cells[i];
            if (c >= 0 && c < d.ncells) d.roots[(int64_t)it.gid * d.ncells + c] = s;
            if (i == 0) {
                const int64_t now = *d.clock;
                d.window[2 * it.gid] = now;
                d.window[2 * it.gid + 1] = now + it.iters;
            }
        }
        return;
    }
    if (w - a.adm_blocks >= a.nwork) return;          // the lone workgroup of an empty update
    const BatchWorkItem &wi = a.w[w - a.adm_blocks];
    for (int i = t; i < wi.nb; i += blockDim.x) {
        const int32_t c = wi.cells[i];
        d.work[wi.off + i] = (c >= 0 && c < d.ncells) ? wi.gid * d.ncells + c : -1;
    }
}

// ---------------------------------------------------------------- particles

__device__ __forceinline__ int bspline(float X, float w[3]) {
    const int base = (int)floorf(X - 0.5f);
    const float fx = X - (float)base;
    const float t0 = 1.5f - fx, t1 = fx - 1.0f, t2 = fx - 0.5f;
    w[0] = 0.5f * (t0 * t0);
    w[1] = 0.75f - t1 * t1;
    w[2] = 0.5f * (t2 * t2);
    return base;
}

// The binned gather works on the nodes [8c - 2, 8c + 9] per axis around root
// cell c (kTile^3 = kTile3): every node touched by a particle whose centre
// node lies in [8c - 1, 8c + 8], i.e. in the block or one node beyond it (a
// particle binned to c that has moved by up to one node since).
constexpr int kTile = 12, kTile3 = 1728;

// s[x * 4 + y * 2 + z] chosen with selects: an array indexed at run time
// would be placed in scratch memory.
__device__ __forceinline__ int32_t pick8(const int32_t s[8], bool x, bool y, bool z) {
    const int32_t a0 = z ? s[1] : s[0], a1 = z ? s[3] : s[2], a2 = z ? s[5] : s[4], a3 = z ? s[7] : s[6];
    const int32_t b0 = y ? a1 : a0, b1 = y ? a3 : a2;
    return x ? b1 : b0;
}

// Gather (G2P) of one particle straight from the grid: v = sum over its 27
// nodes, in (a, b, d) order, of w * node value (0 outside the domain or in an
// inactive block).
template <int KS>
__device__ __forceinline__ void gather_direct(const PartProg &pp, const float x[3], float v[3]) {
    const GridDev &g = pp.gsrc;
    const int N = g.R * kBS;
    float w[3][3];
    int base[3];
    for (int c = 0; c < 3; ++c) base[c] = bspline(x[c] * pp.inv_dx_src, w[c]);
    const float *V0 = chan(g, pp.ch_vsrc), *V1 = chan(g, pp.ch_vsrc + 1), *V2 = chan(g, pp.ch_vsrc + 2);
    // slots of the (at most) 2x2x2 blocks the 27 nodes span, looked up once
    const int blo[3] = {base[0] >> 3, base[1] >> 3, base[2] >> 3};
    int32_t bs[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int ci = blo[0] + (e >> 2), cj = blo[1] + ((e >> 1) & 1), ck = blo[2] + (e & 1);
        const bool in = ci >= 0 && cj >= 0 && ck >= 0 && ci < g.R && cj < g.R && ck < g.R;
        bs[e] = in ? slot_of<KS>(g, ((int64_t)ci * g.R + cj) * g.R + ck) : -1;
    }
    // a row of 3 nodes along k inside one block is read as one 12-byte load per channel
    const bool krow = (base[2] & 7) <= 5 && base[2] >= 0;
    float acc[3] = {0.f, 0.f, 0.f};
    for (int a = 0; a < 3; ++a) {
        const int i = base[0] + a;
        for (int b = 0; b < 3; ++b) {
            const int j = base[1] + b;
            const float wab = w[0][a] * w[1][b];
            const bool ij = i >= 0 && j >= 0 && i < N && j < N;
            float n[3][3];
            if (krow) {
                const int32_t s = ij ? pick8(bs, (i >> 3) != blo[0], (j >> 3) != blo[1], false) : -1;
                float3 r0 = make_float3(0.f, 0.f, 0.f), r1 = r0, r2 = r0;
                if (s >= 0) {
                    const int64_t o = (int64_t)s * kBV + (i & 7) * 64 + (j & 7) * 8 + (base[2] & 7);
                    r0 = *reinterpret_cast<const float3 *>(V0 + o);
                    r1 = *reinterpret_cast<const float3 *>(V1 + o);
                    r2 = *reinterpret_cast<const float3 *>(V2 + o);
                }
                n[0][0] = r0.x; n[1][0] = r0.y; n[2][0] = r0.z;
                n[0][1] = r1.x; n[1][1] = r1.y; n[2][1] = r1.z;
                n[0][2] = r2.x; n[1][2] = r2.y; n[2][2] = r2.z;
            } else {
                for (int d = 0; d < 3; ++d) {
                    const int k = base[2] + d;
                    n[d][0] = n[d][1] = n[d][2] = 0.f;
                    if (ij && k >= 0 && k < N) {
                        const int32_t s = pick8(bs, (i >> 3) != blo[0], (j >> 3) != blo[1], (k >> 3) != blo[2]);
                        if (s >= 0) {
                            const int64_t o = (int64_t)s * kBV + (i & 7) * 64 + (j & 7) * 8 + (k & 7);
                            n[d][0] = V0[o]; n[d][1] = V1[o]; n[d][2] = V2[o];
                        }
                    }
                }
            }
            for (int d = 0; d < 3; ++d) {
                const float wt = wab * w[2][d];
                acc[0] = acc[0] + wt * n[d][0];
                acc[1] = acc[1] + wt * n[d][1];
                acc[2] = acc[2] + wt * n[d][2];
            }
        }
    }
    v[0] = acc[0]; v[1] = acc[1]; v[2] = acc[2];
}

// Scatter (P2G) of one particle straight into the grid with fp32 atomics:
// m += w*m_p, mv_c += (w*m_p)*v_c at each of its 27 nodes inside the domain,
// activating per node, per touched block, or not at all (ACT).
template <int KD, int ACT>
__device__ __forceinline__ void scatter_direct(const PartProg &pp, const int base[3], const float w[3][3],
                                               const float v[3], float mp) {
    const GridDev &g = pp.gdst;
    const int N = g.R * kBS;
    float *M = chan(g, pp.ch_m), *MV0 = chan(g, pp.ch_mv), *MV1 = chan(g, pp.ch_mv + 1), *MV2 = chan(g, pp.ch_mv + 2);
    // per-block activation: the touched nodes span at most 2 blocks per axis
    int32_t bslot[8];
    const int blo[3] = {base[0] >> 3, base[1] >> 3, base[2] >> 3};
    if (ACT == AT_ACT_PER_BLOCK || ACT == AT_ACT_NONE) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int a = e >> 2, b = (e >> 1) & 1, d = e & 1;
            const int ci = blo[0] + a, cj = blo[1] + b, ck = blo[2] + d;
            bslot[e] = -1;
            const bool used = (a == 0 || ((base[0] + 2) >> 3) != blo[0]) &&
                              (b == 0 || ((base[1] + 2) >> 3) != blo[1]) &&
                              (d == 0 || ((base[2] + 2) >> 3) != blo[2]);
            if (!used || ci < 0 || cj < 0 || ck < 0 || ci >= g.R || cj >= g.R || ck >= g.R) continue;
            const int64_t cell = ((int64_t)ci * g.R + cj) * g.R + ck;
            bslot[e] = ACT == AT_ACT_NONE ? slot_of<KD>(g, cell) : activate_cell<KD>(g, cell);
        }
    }
    for (int a = 0; a < 3; ++a) {
        const int i = base[0] + a;
        for (int b = 0; b < 3; ++b) {
            const int j = base[1] + b;
            const float wab = w[0][a] * w[1][b];
            for (int d = 0; d < 3; ++d) {
                const int k = base[2] + d;
                if (i < 0 || j < 0 || k < 0 || i >= N || j >= N || k >= N) continue;
                int32_t s;
                if (ACT == AT_ACT_PER_BLOCK || ACT == AT_ACT_NONE) {
                    s = pick8(bslot, (i >> 3) != blo[0], (j >> 3) != blo[1], (k >> 3) != blo[2]);
                } else {
                    s = activate_cell<KD>(g, ((int64_t)(i >> 3) * g.R + (j >> 3)) * g.R + (k >> 3));
                }
                if (s < 0) continue;
                const int64_t o = (int64_t)s * kBV + (i & 7) * 64 + (j & 7) * 8 + (k & 7);
                const float wt = wab * w[2][d];
                const float tm = wt * mp;
                unsafeAtomicAdd(M + o, tm);
                unsafeAtomicAdd(MV0 + o, tm * v[0]);
                unsafeAtomicAdd(MV1 + o, tm * v[1]);
                unsafeAtomicAdd(MV2 + o, tm * v[2]);
            }
        }
    }
}

// What follows the gather for particle p: advection, then the scatter (or,
// with BIN, its first pass: the root cell of the centre node, base + 1 per
// axis; a particle whose centre node lies outside the domain scatters
// directly and is listed as an outlier of the destination's bins).
template <int KD, uint32_t STEPS, int ACT, bool BIN>
__device__ __forceinline__ void after_gather(const PartProg &pp, int64_t p, float x[3], const float v[3]) {
    const int64_t np = pp.np;
    if (STEPS & PS_ADVECT) {
        for (int c = 0; c < 3; ++c) x[c] = x[c] + pp.dt * v[c];
        pp.x[p] = x[0]; pp.x[np + p] = x[1]; pp.x[2 * np + p] = x[2];
    }
    if (STEPS & PS_P2G) {
        const GridDev &g = pp.gdst;
        const int N = g.R * kBS;
        float w[3][3];
        int base[3];
        for (int c = 0; c < 3; ++c) base[c] = bspline(x[c] * pp.inv_dx_dst, w[c]);
        if (BIN) {
            const int hi = base[0] + 1, hj = base[1] + 1, hk = base[2] + 1;
            if (hi >= 0 && hj >= 0 && hk >= 0 && hi < N && hj < N && hk < N) {
                g.pkr[p] = make_int2(((hi >> 3) * g.R + (hj >> 3)) * g.R + (hk >> 3), 0);
                return;
            }
            g.pkr[p] = make_int2(-1, 0);
            g.pout[atomicAdd(&g.hdr[HDR_NOUT_ACC], 1)] = (int32_t)p;
        }
        scatter_direct<KD, ACT>(pp, base, w, v, pp.m[p]);
    }
}

// One thread per particle: optional gather (G2P), advection and scatter
// (P2G), in index order.
template <int KS, int KD, uint32_t STEPS, int ACT, bool BIN>
__global__ __launch_bounds__(256) void k_particles(PartProg pp) {
    const int64_t np = pp.np;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        float x[3] = {pp.x[p], pp.x[np + p], pp.x[2 * np + p]};
        float v[3];
        if (STEPS & PS_G2P) {
            gather_direct<KS>(pp, x, v);
            pp.v[p] = v[0]; pp.v[np + p] = v[1]; pp.v[2 * np + p] = v[2];
        } else {
            v[0] = pp.v[p]; v[1] = pp.v[np + p]; v[2] = pp.v[2 * np + p];
        }
        after_gather<KD, STEPS, ACT, BIN>(pp, p, x, v);
    }
}

// Gather through the bins of the source grid's last binned scatter (the
// runtime uses them only when that scatter had the same particle count, so
// the bins hold every particle index once; the scatter's outliers are
// listed apart).  The bins may sit in another grid's workspace (gbin_g)
// when that scatter reused them.  Four workgroups per bin (a quarter of its
// particles each) load the tile of the three velocity channels around the
// bin's block (0 outside the domain or in an inactive block) into LDS; each
// particle takes its current position (from its record when the runtime
// knows the records are current, else from x) and, when its 27 nodes lie in
// the tile, gathers from LDS in the same (a, b, d) order and arithmetic as
// gather_direct, so the result is bit-identical.  A particle that has left
// the tile, and every outlier, gathers directly.  When the node's scatter
// reuses these bins, the records are rewritten with the particle's new
// velocity and (advected) position.  Otherwise only v is written: particles
// come in bin order, so the steps that follow a gather in a fused node run
// as a second, index-ordered pass, where their writes stay coalesced.
constexpr int kG2PSplit = 4;   // workgroups per bin (each takes a quarter of its particles)

template <int KS>
__global__ __launch_bounds__(256) void k_g2p_bins(PartProg pp) {
    __shared__ float4 vt[kTile3];   // the three velocity channels of a node side by side
    __shared__ int32_t bsl[27];
    const GridDev &S = pp.gsrc;
    const GridDev &W = pp.gbin_g;
    const int N = S.R * kBS;
    const int64_t np = pp.np;
    const int t = threadIdx.x;
    const int nb = W.hdr[HDR_NBINS];
    const int nout = W.hdr[HDR_NOUT];
    const int nob = (nout + (int)blockDim.x - 1) / (int)blockDim.x;
    const bool advect = (pp.steps & PS_ADVECT) != 0;
    const float *V0 = chan(S, pp.ch_vsrc), *V1 = chan(S, pp.ch_vsrc + 1), *V2 = chan(S, pp.ch_vsrc + 2);
    const int nit = nb * kG2PSplit;
    for (int it = blockIdx.x; it < nit + nob; it += gridDim.x) {
        if (it >= nit) {
            const int q = (it - nit) * (int)blockDim.x + t;
            if (q < nout) {
                const int64_t p = W.pout[q];
                const float x[3] = {pp.x[p], pp.x[np + p], pp.x[2 * np + p]};
                float v[3];
                gather_direct<KS>(pp, x, v);
                pp.v[p] = v[0]; pp.v[np + p] = v[1]; pp.v[2 * np + p] = v[2];
            }
            continue;
        }
        const int4 bin = W.pbins[it / kG2PSplit];
        const int per = (bin.z + kG2PSplit - 1) / kG2PSplit;
        const int q0 = (it % kG2PSplit) * per;
        const int q1 = q0 + per < bin.z ? q0 + per : bin.z;
        if (q0 >= q1) continue;
        int ci, cj, ck;
        cell_coords(W, bin.x, ci, cj, ck);
        const int oi = ci * kBS - 2, oj = cj * kBS - 2, ok = ck * kBS - 2;
        if (t < 27) {
            const int bi = ci - 1 + t / 9, bj = cj - 1 + (t / 3) % 3, bk = ck - 1 + t % 3;
            const bool in = bi >= 0 && bj >= 0 && bk >= 0 && bi < S.R && bj < S.R && bk < S.R;
            bsl[t] = in ? slot_of<KS>(S, ((int64_t)bi * S.R + bj) * S.R + bk) : -1;
        }
        __syncthreads();
        for (int nn = t; nn < kTile3; nn += blockDim.x) {
            const int i = oi + nn / (kTile * kTile), j = oj + (nn / kTile) % kTile, k = ok + nn % kTile;
            float a0 = 0.f, a1 = 0.f, a2 = 0.f;
            if (i >= 0 && j >= 0 && k >= 0 && i < N && j < N && k < N) {
                const int32_t sl = bsl[((i >> 3) - ci + 1) * 9 + ((j >> 3) - cj + 1) * 3 + ((k >> 3) - ck + 1)];
                if (sl >= 0) {
                    const int64_t o = (int64_t)sl * kBV + (i & 7) * 64 + (j & 7) * 8 + (k & 7);
                    a0 = V0[o]; a1 = V1[o]; a2 = V2[o];
                }
            }
            vt[nn] = make_float4(a0, a1, a2, 0.f);
        }
        __syncthreads();
        float4 *const rec = W.pstage + 2 * (int64_t)bin.y;
        for (int q = q0 + t; q < q1; q += blockDim.x) {
            const float4 rb = rec[2 * q + 1];
            const int64_t p = __float_as_int(rb.w);
            float x[3];
            if (pp.g2p_rec_x) {
                const float4 ra = rec[2 * q];
                x[0] = ra.x; x[1] = ra.y; x[2] = ra.z;
            } else {
                x[0] = pp.x[p]; x[1] = pp.x[np + p]; x[2] = pp.x[2 * np + p];
            }
            float w[3][3];
            int base[3];
            for (int c = 0; c < 3; ++c) base[c] = bspline(x[c] * pp.inv_dx_src, w[c]);
            const int ri = base[0] - oi, rj = base[1] - oj, rk = base[2] - ok;
            float v[3];
            if ((unsigned)ri < kTile - 2u && (unsigned)rj < kTile - 2u && (unsigned)rk < kTile - 2u) {
                float acc[3] = {0.f, 0.f, 0.f};
                for (int a = 0; a < 3; ++a) {
                    for (int bb = 0; bb < 3; ++bb) {
                        const float wab = w[0][a] * w[1][bb];
                        const int row = ((ri + a) * kTile + (rj + bb)) * kTile + rk;
                        for (int d = 0; d < 3; ++d) {
                            const float wt = wab * w[2][d];
                            const float4 nv = vt[row + d];
                            acc[0] = acc[0] + wt * nv.x;
                            acc[1] = acc[1] + wt * nv.y;
                            acc[2] = acc[2] + wt * nv.z;
                        }
                    }
                }
                v[0] = acc[0]; v[1] = acc[1]; v[2] = acc[2];
            } else {
                gather_direct<KS>(pp, x, v);
            }
            pp.v[p] = v[0]; pp.v[np + p] = v[1]; pp.v[2 * np + p] = v[2];
            if (pp.p2g_reuse) {
                // the same arithmetic as the index-ordered advection
                if (advect)
                    for (int c = 0; c < 3; ++c) x[c] = x[c] + pp.dt * v[c];
                rec[2 * q] = make_float4(x[0], x[1], x[2], v[0]);
                rec[2 * q + 1] = make_float4(v[1], v[2], rb.z, rb.w);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------ binned scatter (P2G)
// Rank of each binned particle within its cell.  Every particle lands on one
// of the few hundred to thousand cells its grid has active, so counting with
// one global atomic per particle would queue thousands of atomics on each
// counter.  With LDS (root cells <= kHistCells) each workgroup (one per CU)
// counts a contiguous range of particles in an on-chip histogram first and
// adds each cell's total to the global count once, taking its base from the
// returned value.  Whoever takes a cell's count from zero appends the cell to
// the bin list, so the scan only visits non-empty cells.
constexpr int kHistCells = 32768;

__device__ __forceinline__ void append_bin(const GridDev &g, int32_t cell) {
    const int i = atomicAdd(&g.hdr[HDR_NAPPEND], 1);
    g.pbins[i].x = cell;
}

template <bool LDS>
__global__ __launch_bounds__(1024) void k_bin_rank(GridDev g, int64_t np) {
    const int64_t per = (np + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = blockIdx.x * per < np ? blockIdx.x * per : np;
    const int64_t p1 = p0 + per < np ? p0 + per : np;
    const int t = threadIdx.x;
    if (!LDS) {
        for (int64_t p = p0 + t; p < p1; p += blockDim.x) {
            int2 kr = g.pkr[p];
            if (kr.x < 0) continue;
            kr.y = atomicAdd(&g.pcount[kr.x], 1);
            if (kr.y == 0) append_bin(g, kr.x);
            g.pkr[p] = kr;
        }
        return;
    }
    __shared__ int32_t h[kHistCells];
    const int nc = (int)g.ncells;
    for (int c = t; c < nc; c += blockDim.x) h[c] = 0;
    __syncthreads();
    for (int64_t p = p0 + t; p < p1; p += blockDim.x) {
        int2 kr = g.pkr[p];
        if (kr.x < 0) continue;
        kr.y = atomicAdd(&h[kr.x], 1);
        g.pkr[p] = kr;
    }
    __syncthreads();
    for (int c = t; c < nc; c += blockDim.x) {
        const int k = h[c];
        if (k) {
            h[c] = atomicAdd(&g.pcount[c], k);
            if (h[c] == 0) append_bin(g, c);
        }
    }
    __syncthreads();
    for (int64_t p = p0 + t; p < p1; p += blockDim.x) {
        int2 kr = g.pkr[p];
        if (kr.x < 0) continue;
        kr.y += h[kr.x];
        g.pkr[p] = kr;
    }
}

// Exclusive scan, in one workgroup, of the counts of the non-empty cells
// (in the order they were appended): each bin's first position, the final
// bin list {cell, first, count, 0} and its length; the counts and the append
// counter are cleared for the next scatter.
__global__ __launch_bounds__(1024) void k_bin_scan(GridDev g) {
    __shared__ int wsum[16];
    const int n = g.hdr[HDR_NAPPEND];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int per = (n + 1023) / 1024;
    const int i0 = t * per < n ? t * per : n;
    const int i1 = i0 + per < n ? i0 + per : n;
    int cnt = 0;
    for (int i = i0; i < i1; ++i) cnt += g.pcount[g.pbins[i].x];
    const int ic = wave_incl_scan(cnt);
    if (lane == 63) wsum[wid] = ic;
    __syncthreads();
    int pos = ic - cnt;
    for (int w = 0; w < wid; ++w) pos += wsum[w];
    for (int i = i0; i < i1; ++i) {
        const int32_t c = g.pbins[i].x;
        const int k = g.pcount[c];
        g.poff[c] = pos;
        g.pbins[i] = make_int4(c, pos, k, 0);
        pos += k;
        g.pcount[c] = 0;
    }
    __syncthreads();
    if (t == 0) {
        g.hdr[HDR_NBINS] = n;
        g.hdr[HDR_NAPPEND] = 0;
        g.hdr[HDR_NOUT] = g.hdr[HDR_NOUT_ACC];
        g.hdr[HDR_NOUT_ACC] = 0;
    }
}

// Particle records grouped by cell: record poff[cell] + rank holds the
// particle's x, v, m and index (read in index order, written as two float4),
// so a bin's particles are read contiguously by the tile kernels.
__global__ __launch_bounds__(256) void k_bin_place(PartProg pp) {
    const GridDev &g = pp.gdst;
    const int64_t np = pp.np;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        const int2 kr = g.pkr[p];
        if (kr.x < 0) continue;
        const int64_t pos = (int64_t)g.poff[kr.x] + kr.y;
        g.pstage[2 * pos] = make_float4(pp.x[p], pp.x[np + p], pp.x[2 * np + p], pp.v[p]);
        g.pstage[2 * pos + 1] = make_float4(pp.v[np + p], pp.v[2 * np + p], pp.m[p], __int_as_float((int32_t)p));
    }
}

// Sort key of a centre node at offset (a, b, c) in [0, 9]^3 from 8 x cell - 1
// (the bin's block is [1, 8]^3): the 512 nodes inside the block first, in
// (a, b, c) order, then the 488 around it (the two a-faces, then the two
// b-faces, then the two c-faces of what is left).  centre_of_key inverts it.
__device__ __forceinline__ int centre_key(int a, int b, int c) {
    const bool ia = a >= 1 && a <= 8, ib = b >= 1 && b <= 8, ic = c >= 1 && c <= 8;
    if (ia && ib && ic) return ((a - 1) * 8 + (b - 1)) * 8 + (c - 1);
    if (!ia) return 512 + (a == 9 ? 100 : 0) + b * 10 + c;
    if (!ib) return 712 + (a - 1) * 20 + (b == 9 ? 10 : 0) + c;
    return 872 + (a - 1) * 16 + (b - 1) * 2 + (c == 9 ? 1 : 0);
}

__device__ __forceinline__ void centre_of_key(int key, int &a, int &b, int &c) {
    if (key < 512) {
        a = 1 + (key >> 6); b = 1 + ((key >> 3) & 7); c = 1 + (key & 7);
        return;
    }
    int h = key - 512;
    if (h < 200) {
        a = h < 100 ? 0 : 9; b = (h % 100) / 10; c = h % 10;
        return;
    }
    h -= 200;
    if (h < 160) {
        a = 1 + h / 20; b = (h % 20) < 10 ? 0 : 9; c = h % 10;
        return;
    }
    h -= 160;
    a = 1 + h / 16; b = 1 + (h % 16) / 2; c = (h & 1) ? 9 : 0;
}

// One workgroup per bin (root cell c) of the bins in gbin_s (the
// destination's own, just made, or reused ones whose records the node's
// gather has brought up to date).  The nodes a bin's particles touch form a
// tile held in LDS with the four channels (m, mv) of a node side by side:
// [8c - 1, 8c + 8] per axis for bins just made (every centre node lies in
// the block), [8c - 2, 8c + 9] when WIDE, for reused bins, whose particles
// may have moved one node past the block (one further, they scatter
// directly).  The bin's particles (in chunks) are first counting-sorted by
// centre node (integer LDS atomics).  Each thread then owns one centre node
// per round (rounds of 256; a round with no particles in the workgroup is
// skipped) and sums, in registers, the contributions of its particles to the
// 27 nodes around it (the direct scatter's contributions, with the mass
// folded into the k-weights and fused multiply-adds: rounding differs within
// the scatter's summation bound).  The sums reach the tile in 27 phases, one per node offset,
// separated by barriers: within a phase distinct centre nodes add to
// distinct tile nodes, so each add is a plain LDS read and write (LDS float
// atomics are slow on this hardware) and the tile's summation order is
// fixed.  The touched blocks among the 27 around c are activated (or were,
// per node, when ACT == AT_ACT_PER_NODE) and the tile's non-zero values are
// added to the grid with one global atomic per node and channel.  When
// reusing, workgroups past the bins scatter the outliers listed with the
// bins directly, from the particle arrays.

template <int KD, int ACT, bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_p2g_bins(PartProg pp) {
    constexpr int TE = WIDE ? 12 : 10, T3 = TE * TE * TE;   // tile edge and nodes
    constexpr int HALO = WIDE ? 2 : 1;                       // tile origin 8c - HALO
    constexpr int NC = WIDE ? 10 : 8;                        // centre-node range edge, from 8c - HALO + 1
    constexpr int KEYS = WIDE ? 1024 : 512, KPT = KEYS / 256; // sort keys (wide: 1000 padded), per thread
    constexpr int CHUNK = 4096;
    __shared__ float4 tile[T3];
    __shared__ int32_t tslot[27];
    __shared__ int32_t tflag[27];
    __shared__ int32_t ncnt[KEYS];       // particles per centre-node key; then first, then one-past-last position
    __shared__ int32_t wsum[4];
    __shared__ int32_t nhalo;            // wide: non-empty keys outside the block
    __shared__ int32_t chist[64];        // block centre nodes per particle count (capped), then first rank
    __shared__ int16_t byload[512];      // block centre nodes by decreasing particle count
    __shared__ int16_t hkeys[WIDE ? 488 : 1];
    __shared__ uint16_t order[CHUNK];    // chunk-relative particle index, sorted by centre node
    // narrow: key << 16 | rank among the chunk's particles there (-1: direct);
    // wide tiles have no room for it and place by a second pass of keys
    __shared__ int32_t lrank[WIDE ? 1 : CHUNK];
    const GridDev &g = pp.gdst;
    const GridDev &W = pp.gbin_s;
    const int N = g.R * kBS;
    const int nbins = W.hdr[HDR_NBINS];
    const int nout = pp.p2g_reuse ? W.hdr[HDR_NOUT] : 0;
    const int nob = (nout + (int)blockDim.x - 1) / (int)blockDim.x;
    const int64_t np = pp.np;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    float *const M = chan(g, pp.ch_m), *const MV0 = chan(g, pp.ch_mv), *const MV1 = chan(g, pp.ch_mv + 1),
                 *const MV2 = chan(g, pp.ch_mv + 2);
    for (int b = blockIdx.x; b < nbins + nob; b += gridDim.x) {
        if (b >= nbins) {
            const int q = (b - nbins) * (int)blockDim.x + t;
            if (q < nout) {
                const int64_t p = W.pout[q];
                const float x[3] = {pp.x[p], pp.x[np + p], pp.x[2 * np + p]};
                const float v[3] = {pp.v[p], pp.v[np + p], pp.v[2 * np + p]};
                float w[3][3];
                int base[3];
                for (int c = 0; c < 3; ++c) base[c] = bspline(x[c] * pp.inv_dx_dst, w[c]);
                scatter_direct<KD, ACT>(pp, base, w, v, pp.m[p]);
            }
            continue;
        }
        const int4 bin = W.pbins[b];
        int ci, cj, ck;
        cell_coords(W, bin.x, ci, cj, ck);
        const int oi = ci * kBS - HALO, oj = cj * kBS - HALO, ok = ck * kBS - HALO;
        for (int q = t; q < T3; q += blockDim.x) tile[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (t < 27) tflag[t] = 0;
        // sort key of particle q's centre node (base + 1 per axis, as an
        // offset in [0, NC) from 8c - HALO + 1), or -1 when it does not fit
        // the tile
        auto key_of = [&](const float4 &ra) {
            const int ha = (int)floorf(ra.x * pp.inv_dx_dst - 0.5f) + HALO - ci * kBS;
            const int hb = (int)floorf(ra.y * pp.inv_dx_dst - 0.5f) + HALO - cj * kBS;
            const int hc = (int)floorf(ra.z * pp.inv_dx_dst - 0.5f) + HALO - ck * kBS;
            if ((unsigned)ha >= (unsigned)NC || (unsigned)hb >= (unsigned)NC || (unsigned)hc >= (unsigned)NC) return -1;
            return WIDE ? centre_key(ha, hb, hc) : (ha * 8 + hb) * 8 + hc;
        };
        for (int c0 = 0; c0 < bin.z; c0 += CHUNK) {
            const int n = bin.z - c0 < CHUNK ? bin.z - c0 : CHUNK;
            const float4 *const rec = W.pstage + 2 * ((int64_t)bin.y + c0);
            for (int q = t; q < KEYS; q += blockDim.x) ncnt[q] = 0;
            if (t == 0) nhalo = 0;
            __syncthreads();
            // count per centre node; a particle that does not fit the tile
            // scatters directly
            for (int q = t; q < n; q += blockDim.x) {
                const float4 ra = rec[2 * q];
                const int key = key_of(ra);
                if (key >= 0) {
                    if constexpr (WIDE)
                        atomicAdd(&ncnt[key], 1);
                    else
                        lrank[q] = (key << 16) | atomicAdd(&ncnt[key], 1);
                } else {
                    if constexpr (!WIDE) lrank[q] = -1;
                    const float4 rb = rec[2 * q + 1];
                    const float x[3] = {ra.x, ra.y, ra.z};
                    const float v[3] = {ra.w, rb.x, rb.y};
                    float w[3][3];
                    int base[3];
                    for (int c = 0; c < 3; ++c) base[c] = bspline(x[c] * pp.inv_dx_dst, w[c]);
                    scatter_direct<KD, ACT>(pp, base, w, v, rb.z);
                }
            }
            __syncthreads();
            // scan of the counts (KPT consecutive keys per thread): narrow
            // keeps each key's end, wide its start (placement advances it to
            // the end) and lists the non-empty keys outside the block
            int cnt[KPT], tot = 0;
#pragma unroll
            for (int e = 0; e < KPT; ++e) tot += (cnt[e] = ncnt[KPT * t + e]);
            const int incl = wave_incl_scan(tot);
            if (lane == 63) wsum[wid] = incl;
            __syncthreads();
            int before = incl - tot;
            for (int w = 0; w < wid; ++w) before += wsum[w];
#pragma unroll
            for (int e = 0; e < KPT; ++e) {
                ncnt[KPT * t + e] = WIDE ? before : before + cnt[e];
                before += cnt[e];
                if (WIDE && KPT * t + e >= 512 && cnt[e] > 0) hkeys[atomicAdd(&nhalo, 1)] = (int16_t)(KPT * t + e);
            }
            __syncthreads();
            if constexpr (WIDE) {
                for (int q = t; q < n; q += blockDim.x) {
                    const int key = key_of(rec[2 * q]);
                    if (key >= 0) order[atomicAdd(&ncnt[key], 1)] = (uint16_t)q;
                }
            } else {
                for (int q = t; q < n; q += blockDim.x) {
                    const int lr = lrank[q];
                    if (lr < 0) continue;
                    const int key = lr >> 16;
                    order[(key > 0 ? ncnt[key - 1] : 0) + (lr & 0xffff)] = (uint16_t)q;
                }
            }
            __syncthreads();
            // one round: each thread sums the particles of centre-node key
            // `own` (none when own < 0) and adds the sums to the tile
            auto round = [&](int own) {
                const int p0 = own > 0 ? ncnt[own - 1] : 0;
                const int pe = own >= 0 ? ncnt[own] : 0;
                const bool any = p0 < pe;
                int la = 0, lb = 0, lc = 0;
                if (any) {
                    if (WIDE) {
                        centre_of_key(own, la, lb, lc);
                    } else {
                        la = own >> 6; lb = (own >> 3) & 7; lc = own & 7;
                    }
                }
                float acc[27][4];
#pragma unroll
                for (int e = 0; e < 27; ++e) acc[e][0] = acc[e][1] = acc[e][2] = acc[e][3] = 0.f;
                // the next particle's record is loaded while the current one is summed
                float4 na = make_float4(0.f, 0.f, 0.f, 0.f), nb = na;
                if (any) {
                    const int q = order[p0];
                    na = rec[2 * q];
                    nb = rec[2 * q + 1];
                }
                for (int pos = p0; pos < pe; ++pos) {
                    const float4 ra = na, rb = nb;
                    const int q = order[pos + 1 < pe ? pos + 1 : pos];
                    na = rec[2 * q];
                    nb = rec[2 * q + 1];
                    const float x[3] = {ra.x, ra.y, ra.z};
                    const float v[3] = {ra.w, rb.x, rb.y};
                    const float mp = rb.z;
                    float w[3][3];
                    int base[3];
                    for (int c = 0; c < 3; ++c) base[c] = bspline(x[c] * pp.inv_dx_dst, w[c]);
                    // the mass folded into the k-weights and fused multiply-adds:
                    // these sums only have to meet the scatter's summation bound,
                    // and they are what bounds this kernel (vector ALU)
                    const float wkm[3] = {w[2][0] * mp, w[2][1] * mp, w[2][2] * mp};
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
#pragma unroll
                        for (int bb = 0; bb < 3; ++bb) {
                            const float wab = w[0][a] * w[1][bb];
#pragma unroll
                            for (int d = 0; d < 3; ++d) {
                                if (ACT == AT_ACT_PER_NODE) {
                                    const int i = base[0] + a, j = base[1] + bb, kk = base[2] + d;
                                    if (i >= 0 && j >= 0 && kk >= 0 && i < N && j < N && kk < N)
                                        activate_cell<KD>(g, ((int64_t)(i >> 3) * g.R + (j >> 3)) * g.R + (kk >> 3));
                                }
                                const float tm = wab * wkm[d];
                                float *s4 = acc[(a * 3 + bb) * 3 + d];
                                s4[0] = s4[0] + tm;
                                s4[1] = __builtin_fmaf(tm, v[0], s4[1]);
                                s4[2] = __builtin_fmaf(tm, v[1], s4[2]);
                                s4[3] = __builtin_fmaf(tm, v[2], s4[3]);
                            }
                        }
                    }
                }
                // node offset e = (a * 3 + b) * 3 + d of centre (la, lb, lc)
                // is tile node (la + a, lb + b, lc + d)
#pragma unroll
                for (int e = 0; e < 27; ++e) {
                    __syncthreads();
                    const int a = e / 9, bb = (e / 3) % 3, d = e % 3;
                    const int i = oi + la + a, j = oj + lb + bb, kk = ok + lc + d;
                    if (any && i >= 0 && j >= 0 && kk >= 0 && i < N && j < N && kk < N) {
                        const int nn = ((la + a) * TE + (lb + bb)) * TE + (lc + d);
                        float4 cur = tile[nn];
                        cur.x = cur.x + acc[e][0];
                        cur.y = cur.y + acc[e][1];
                        cur.z = cur.z + acc[e][2];
                        cur.w = cur.w + acc[e][3];
                        tile[nn] = cur;
                        tflag[((i >> 3) - ci + 1) * 9 + ((j >> 3) - cj + 1) * 3 + ((kk >> 3) - ck + 1)] = 1;
                    }
                }
            };
            // the block's 512 centre nodes go to threads by decreasing
            // particle count (any assignment keeps a phase's targets
            // distinct), so a wave's lanes run loops of similar length; then
            // the listed nodes around the block
            if (t < 64) chist[t] = 0;
            __syncthreads();
            int load[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int key = 2 * t + h;
                load[h] = min(ncnt[key] - (key > 0 ? ncnt[key - 1] : 0), 63);
                atomicAdd(&chist[load[h]], 1);
            }
            __syncthreads();
            if (t == 0) {
                int run = 0;
                for (int q = 63; q >= 0; --q) {
                    const int c = chist[q];
                    chist[q] = run;
                    run += c;
                }
            }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h) byload[atomicAdd(&chist[load[h]], 1)] = (int16_t)(2 * t + h);
            __syncthreads();
            for (int r = 0; r < 2; ++r) {
                const int own = byload[r * 256 + t];
                if (__syncthreads_or(ncnt[own] > (own > 0 ? ncnt[own - 1] : 0))) round(own);
            }
            if (WIDE)
                for (int h0 = 0; h0 < nhalo; h0 += 256) round(h0 + t < nhalo ? hkeys[h0 + t] : -1);
            __syncthreads();
        }
        if (t < 27) {
            int32_t sl = -1;
            if (tflag[t]) {
                const int64_t cell = ((int64_t)(ci - 1 + t / 9) * g.R + (cj - 1 + (t / 3) % 3)) * g.R + (ck - 1 + t % 3);
                // already active under per-node activation; looked up only under none
                sl = ACT == AT_ACT_NONE ? slot_of<KD>(g, cell) : activate_cell<KD>(g, cell);
            }
            tslot[t] = sl;
        }
        __syncthreads();
        for (int nn = t; nn < T3; nn += blockDim.x) {
            const int i = oi + nn / (TE * TE), j = oj + (nn / TE) % TE, k = ok + nn % TE;
            if (i < 0 || j < 0 || k < 0 || i >= N || j >= N || k >= N) continue;
            const int32_t sl = tslot[((i >> 3) - ci + 1) * 9 + ((j >> 3) - cj + 1) * 3 + ((k >> 3) - ck + 1)];
            if (sl < 0) continue;
            const int64_t o = (int64_t)sl * kBV + (i & 7) * 64 + (j & 7) * 8 + (k & 7);
            const float4 tv = tile[nn];
            if (tv.x != 0.f) unsafeAtomicAdd(M + o, tv.x);
            if (tv.y != 0.f) unsafeAtomicAdd(MV0 + o, tv.y);
            if (tv.z != 0.f) unsafeAtomicAdd(MV1 + o, tv.z);
            if (tv.w != 0.f) unsafeAtomicAdd(MV2 + o, tv.w);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- setup/inspection

template <int KIND>
__global__ __launch_bounds__(kSFThreads) void k_scatter_blocks(GridDev g, int ch, const int32_t *cells,
                                                                const float *vals, int64_t n) {
    for (int64_t e = blockIdx.x; e < n; e += gridDim.x) {
        const int32_t cell = cells[e];
        if (cell < 0 || cell >= g.ncells) continue;
        const int32_t s = activate_cell<KIND>(g, cell);
        if (s < 0) continue;
        reinterpret_cast<float4 *>(chan(g, ch) + (int64_t)s * kBV)[threadIdx.x] =
            reinterpret_cast<const float4 *>(vals + e * kBV)[threadIdx.x];
    }
}

template <int KIND>
__global__ __launch_bounds__(kSFThreads) void k_gather_blocks(GridDev g, int ch, const int32_t *cells,
                                                               float *vals, int64_t n) {
    for (int64_t e = blockIdx.x; e < n; e += gridDim.x) {
        const int32_t cell = cells[e];
        const int32_t s = (cell >= 0 && cell < g.ncells) ? slot_of<KIND>(g, cell) : -1;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (s >= 0) v = reinterpret_cast<const float4 *>(chan(g, ch) + (int64_t)s * kBV)[threadIdx.x];
        reinterpret_cast<float4 *>(vals + e * kBV)[threadIdx.x] = v;
    }
}

// hdr[HDR_SCRATCH] = popcount of the activity bits (one workgroup, no
// pre-clear needed).
__global__ __launch_bounds__(1024) void k_popcount(GridDev g) {
    __shared__ int wsum[16];
    const int64_t W = (g.ncells + 31) >> 5;
    const uint32_t tail = (g.ncells & 31) ? ((1u << (g.ncells & 31)) - 1u) : 0xffffffffu;
    int cnt = 0;
    for (int64_t w = threadIdx.x; w < W; w += blockDim.x) {
        uint32_t b = g.bits[w];
        if (w == W - 1) b &= tail;
        cnt += __popc(b);
    }
    const int incl = wave_incl_scan(cnt);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int q = 0; q < (int)((blockDim.x + 63) >> 6); ++q) s += wsum[q];
        g.hdr[HDR_SCRATCH] = s;
    }
}

// Clears what the binning kernels expect to find at zero before a scatter
// that bins through the static workspace: the per-cell counts of the cells
// it may touch and the grid's append and outlier counters (a plain kernel,
// not a memset, so that the clear can sit in a captured graph).
__global__ __launch_bounds__(256) void k_static_clear(int32_t *pcount, int64_t n, int32_t *hdr) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pcount[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hdr[HDR_NAPPEND] = 0;
        hdr[HDR_NOUT_ACC] = 0;
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers

int struct_for_grid_size(const GridDev &g) {
    if (g_sf_grid_override > 0) return g_sf_grid_override;
    // persistent grid: enough workgroups to fill 256 CUs several times over,
    // never more than the list can hold; a multiple of 8 (one slice per XCD)
    const int64_t cap = g.cap < g.ncells ? g.cap : g.ncells;
    int64_t wg = 256 * 8;
    if (cap < wg) wg = ((cap + 7) / 8) * 8;
    if (wg < 8) wg = 8;
    return (int)wg;
}

// Wavefront-per-block kernels.  The software-pipelined forms want several
// blocks per wavefront (7 resident wavefronts per CU measured best on the
// 13k-block band: 4, 5, 6, 8, 12 and 16 were slower); the direct forms hide
// latency with occupancy instead.
int wave_grid_size(const GridDev &g, bool pipelined) {
    if (g_sf_grid_override > 0) return g_sf_grid_override;
    const int64_t cap = g.cap < g.ncells ? g.cap : g.ncells;
    int64_t wg = pipelined ? 256 * 7 : 256 * 28;
    if (cap < wg) wg = ((cap + 7) / 8) * 8;
    if (wg < 8) wg = 8;
    return (int)wg;
}

void set_struct_for_grid_size(int wgs) { g_sf_grid_override = wgs > 0 ? ((wgs + 7) / 8) * 8 : 0; }

int struct_for_kernel() { return g_sf_kernel; }
int struct_for_grid_size_override() { return g_sf_grid_override; }
int batch_waves() { return g_batch_waves; }
void set_batch_waves(int waves) { g_batch_waves = waves; }
void set_struct_for_kernel(int form) { g_sf_kernel = form; }

hipError_t launch_activate(const GridDev &g, const int32_t *ijk, int64_t n, int coord_kind, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 65536) blocks = 65536;
    if (g.kind == AT_ROOT_BITMASK)
        hipLaunchKernelGGL(k_activate<AT_ROOT_BITMASK>, dim3((unsigned)blocks), dim3(256), 0, s, g, ijk, n, coord_kind);
    else
        hipLaunchKernelGGL(k_activate<AT_ROOT_POINTER>, dim3((unsigned)blocks), dim3(256), 0, s, g, ijk, n, coord_kind);
    return hipGetLastError();
}

template <int KIND>
static void launch_listgen_k(const GridDev &g, uint64_t *flags, uint32_t epoch, hipStream_t s) {
    int64_t C = 8;
    while ((g.ncells + 256 * C - 1) / (256 * C) > kScanMaxWG) C *= 2;
    const unsigned blocks = (unsigned)((g.ncells + 256 * C - 1) / (256 * C));
    if (C == 8 && (g.ncells + 31) / 32 <= kPrefixWords) {
        hipLaunchKernelGGL((k_listgen<KIND, 8, true>), dim3(blocks), dim3(256), 0, s, g, flags, epoch);
        return;
    }
    switch (C) {
    case 8: hipLaunchKernelGGL((k_listgen<KIND, 8, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    case 16: hipLaunchKernelGGL((k_listgen<KIND, 16, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    case 32: hipLaunchKernelGGL((k_listgen<KIND, 32, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    case 64: hipLaunchKernelGGL((k_listgen<KIND, 64, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    case 128: hipLaunchKernelGGL((k_listgen<KIND, 128, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    case 256: hipLaunchKernelGGL((k_listgen<KIND, 256, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    case 512: hipLaunchKernelGGL((k_listgen<KIND, 512, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    case 1024: hipLaunchKernelGGL((k_listgen<KIND, 1024, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    case 2048: hipLaunchKernelGGL((k_listgen<KIND, 2048, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    default: hipLaunchKernelGGL((k_listgen<KIND, 4096, false>), dim3(blocks), dim3(256), 0, s, g, flags, epoch); break;
    }
}

hipError_t launch_listgen(const GridDev &g, uint64_t *flags, uint32_t epoch, hipStream_t s) {
    if (g.kind == AT_ROOT_BITMASK) launch_listgen_k<AT_ROOT_BITMASK>(g, flags, epoch, s);
    else launch_listgen_k<AT_ROOT_POINTER>(g, flags, epoch, s);
    return hipGetLastError();
}

template <int OP, int KIND, bool CHECK>
static void launch_stencil_c(const GridDev &g, const StencilCh &c, float p, int table, hipStream_t s) {
    const dim3 grid(wave_grid_size(g, table && g_sf_kernel == 0)), block(64);
    if (table && g_sf_kernel == 0 && kStencilLds && (OP == AT_OP_LAP_UPDATE || OP == AT_OP_JACOBI))
        hipLaunchKernelGGL((k_stencil_lds<OP, CHECK, KIND>), grid, block, 0, s, g, (const int32_t *)g.list, c, p);
    else if (table && g_sf_kernel == 0)
        hipLaunchKernelGGL((k_stencil_pipe<OP, KIND, CHECK>), grid, block, 0, s, g, (const int32_t *)g.list, c, p);
    else if (table && g_sf_kernel == 1)
        hipLaunchKernelGGL((k_stencil<OP, KIND, CHECK, true>), grid, block, 0, s, g, c, p);
    else
        hipLaunchKernelGGL((k_stencil<OP, KIND, CHECK, false>), grid, block, 0, s, g, c, p);
}

template <int OP, int KIND>
static void launch_stencil_t(const GridDev &g, const StencilCh &c, float p, int check, int table, hipStream_t s) {
    if (check) launch_stencil_c<OP, KIND, true>(g, c, p, table, s);
    else launch_stencil_c<OP, KIND, false>(g, c, p, table, s);
}

template <int OP>
static void launch_stencil_k(const GridDev &g, const StencilCh &c, float p, int check, int table, hipStream_t s) {
    if (g.kind == AT_ROOT_BITMASK) launch_stencil_t<OP, AT_ROOT_BITMASK>(g, c, p, check, table, s);
    else launch_stencil_t<OP, AT_ROOT_POINTER>(g, c, p, check, table, s);
}

hipError_t launch_stencil(const GridDev &g, int op, const int32_t *ch, float p, int check, int table, hipStream_t s) {
    StencilCh c{};
    auto C = [&](int i) { return g.chan + (int64_t)ch[i] * g.ch_stride; };
    switch (op) {
    case AT_OP_LAP_UPDATE:
        c.tin[0] = C(0); c.out0 = C(1);
        launch_stencil_k<AT_OP_LAP_UPDATE>(g, c, p, check, table, s);
        break;
    case AT_OP_JACOBI:
        c.tin[0] = C(0); c.ein = C(1); c.out0 = C(2);
        launch_stencil_k<AT_OP_JACOBI>(g, c, p, check, table, s);
        break;
    case AT_OP_DIFFUSE:
        c.tin[0] = C(0); c.tin[1] = C(1); c.out0 = C(2);
        launch_stencil_k<AT_OP_DIFFUSE>(g, c, p, check, table, s);
        break;
    case AT_OP_DIFFUSE_ADJ:
        c.tin[0] = C(0); c.tin[1] = C(1); c.tin[2] = C(2); c.out0 = C(3); c.ein = C(4); c.out1 = C(4);
        launch_stencil_k<AT_OP_DIFFUSE_ADJ>(g, c, p, check, table, s);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND, bool CHECK>
static bool launch_elem_k(const GridDev &g, const MicroOp &op, dim3 grid, hipStream_t s) {
    const int32_t *recs = g.list;
    switch (op.op) {
    case AT_OP_COPY: hipLaunchKernelGGL((k_elem<AT_OP_COPY, KIND, CHECK>), grid, dim3(64), 0, s, g, recs, op); return true;
    case AT_OP_AXPY: hipLaunchKernelGGL((k_elem<AT_OP_AXPY, KIND, CHECK>), grid, dim3(64), 0, s, g, recs, op); return true;
    case AT_OP_INC: hipLaunchKernelGGL((k_elem<AT_OP_INC, KIND, CHECK>), grid, dim3(64), 0, s, g, recs, op); return true;
    case AT_OP_FILL: hipLaunchKernelGGL((k_elem<AT_OP_FILL, KIND, CHECK>), grid, dim3(64), 0, s, g, recs, op); return true;
    case AT_OP_NORMALISE:
        hipLaunchKernelGGL((k_elem<AT_OP_NORMALISE, KIND, CHECK>), grid, dim3(64), 0, s, g, recs, op);
        return true;
    case AT_OP_MPM_GRID:
        hipLaunchKernelGGL((k_elem<AT_OP_MPM_GRID, KIND, CHECK>), grid, dim3(64), 0, s, g, recs, op);
        return true;
    default: return false;
    }
}

bool tail_op_supported(int op) {
    return op == AT_OP_AXPY || op == AT_OP_INC || op == AT_OP_COPY || op == AT_OP_FILL;
}

template <int OP>
static void launch_tail_k(const GridDev &g, const StencilCh &c, float p, const MicroProg &tail, int out_ch,
                          int in_ch, hipStream_t s) {
    const dim3 grid(wave_grid_size(g, true)), block(64);
    if constexpr (OP == AT_OP_JACOBI || OP == AT_OP_LAP_UPDATE) {
        if (kStencilLds) {
            hipLaunchKernelGGL((k_stencil_tail_lds<OP>), grid, block, 0, s, g, (const int32_t *)g.list, c, p, tail,
                               out_ch, in_ch);
            return;
        }
    }
    if (g.kind == AT_ROOT_BITMASK)
        hipLaunchKernelGGL((k_stencil_tail<OP, AT_ROOT_BITMASK>), grid, block, 0, s, g, (const int32_t *)g.list, c, p,
                           tail, out_ch, in_ch);
    else
        hipLaunchKernelGGL((k_stencil_tail<OP, AT_ROOT_POINTER>), grid, block, 0, s, g, (const int32_t *)g.list, c, p,
                           tail, out_ch, in_ch);
}

hipError_t launch_stencil_tail(const GridDev &g, int op, const int32_t *ch, float p, const MicroProg &tail,
                               hipStream_t s) {
    StencilCh c{};
    auto C = [&](int i) { return g.chan + (int64_t)ch[i] * g.ch_stride; };
    switch (op) {
    case AT_OP_LAP_UPDATE:
        c.tin[0] = C(0); c.out0 = C(1);
        launch_tail_k<AT_OP_LAP_UPDATE>(g, c, p, tail, ch[1], ch[0], s);
        break;
    case AT_OP_JACOBI:
        c.tin[0] = C(0); c.ein = C(1); c.out0 = C(2);
        launch_tail_k<AT_OP_JACOBI>(g, c, p, tail, ch[2], ch[0], s);
        break;
    case AT_OP_DIFFUSE:
        c.tin[0] = C(0); c.tin[1] = C(1); c.out0 = C(2);
        launch_tail_k<AT_OP_DIFFUSE>(g, c, p, tail, ch[2], ch[0], s);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND, int NT>
static void launch_tile_nt(const GridDev &g, const TileProg &tp, dim3 grid, size_t lds, hipStream_t s) {
    if (tp.vstage) hipLaunchKernelGGL((k_tile_micro<KIND, NT, true>), grid, dim3(kTT), lds, s, g, tp);
    else hipLaunchKernelGGL((k_tile_micro<KIND, NT, false>), grid, dim3(kTT), lds, s, g, tp);
}

template <int KIND>
static void launch_tile_k(const GridDev &g, const TileProg &tp, dim3 grid, size_t lds, hipStream_t s) {
    switch (tp.nt) {
    case 1: launch_tile_nt<KIND, 1>(g, tp, grid, lds, s); break;
    case 2: launch_tile_nt<KIND, 2>(g, tp, grid, lds, s); break;
    case 3: launch_tile_nt<KIND, 3>(g, tp, grid, lds, s); break;
    default: launch_tile_nt<KIND, 4>(g, tp, grid, lds, s); break;
    }
}

// A node for k_tile_micro: no activation check; sampling ops (ADVECT,
// MACCORMACK) with element-wise ops it implements (COPY, AXPY, INC, FILL);
// at most kTileCh distinct sampled channels; RK3 ops sharing one velocity.
bool tile_prog(const MicroProg &prog, TileProg &tp) {
    if (prog.check || prog.verify || g_sf_kernel != 0) return false;
    tp = TileProg{};
    tp.prog = prog;
    tp.v0 = -1;
    bool sampling = false, shared_v = true;
    for (int o = 0; o < prog.nops; ++o) {
        const MicroOp &op = prog.ops[o];
        if (op.op == AT_OP_ADVECT || op.op == AT_OP_MACCORMACK) {
            bool have = false;
            for (int q = 0; q < tp.nt; ++q) have |= tp.tch[q] == op.ch[0];
            if (!have) {
                if (tp.nt == kTileCh) return false;
                tp.tch[tp.nt++] = op.ch[0];
            }
            if (sampling && op.ch[1] != tp.v0) shared_v = false;
            if (!sampling) tp.v0 = op.ch[1];
            if (op.p1 != 0.f) tp.vstage = 1;
            sampling = true;
        } else if (op.op != AT_OP_COPY && op.op != AT_OP_AXPY && op.op != AT_OP_INC && op.op != AT_OP_FILL) {
            return false;
        }
    }
    // RK3 back-traces sample one staged velocity; else each op reads its own
    if (!shared_v) {
        if (tp.vstage) return false;
        tp.v0 = -1;
    }
    return sampling;
}

size_t tile_lds_bytes(const TileProg &tp) { return (size_t)tile_lds_floats(tp) * sizeof(float); }

unsigned tile_grid_size(const GridDev &g, size_t lds) {
    const int64_t cap = g.cap < g.ncells ? g.cap : g.ncells;
    // as many resident workgroups as the CU's 160 KiB of LDS holds (at most 8)
    int64_t per_cu = (int64_t)(160 * 1024) / (int64_t)(lds + 256);
    if (per_cu > 8) per_cu = 8;
    if (per_cu < 1) per_cu = 1;
    int64_t wgs = 256 * per_cu;
    if (cap < wgs) wgs = ((cap + 7) / 8) * 8;
    return (unsigned)wgs;
}

hipError_t launch_micro(const GridDev &g, const MicroProg &prog, hipStream_t s) {
    TileProg tp;
    if (tile_prog(prog, tp)) {
        const size_t lds = tile_lds_bytes(tp);
        const dim3 grid(tile_grid_size(g, lds));
        if (g.kind == AT_ROOT_BITMASK) launch_tile_k<AT_ROOT_BITMASK>(g, tp, grid, lds, s);
        else launch_tile_k<AT_ROOT_POINTER>(g, tp, grid, lds, s);
        return hipGetLastError();
    }
    const dim3 grid(wave_grid_size(g, false)), block(64);
    if (prog.nops == 1 && g_sf_kernel == 0 && !prog.verify) {
        const dim3 pgrid(wave_grid_size(g, true));
        // a single element-wise op runs the pipelined kernel
        bool done;
        if (g.kind == AT_ROOT_BITMASK)
            done = prog.check ? launch_elem_k<AT_ROOT_BITMASK, true>(g, prog.ops[0], pgrid, s)
                              : launch_elem_k<AT_ROOT_BITMASK, false>(g, prog.ops[0], pgrid, s);
        else
            done = prog.check ? launch_elem_k<AT_ROOT_POINTER, true>(g, prog.ops[0], pgrid, s)
                              : launch_elem_k<AT_ROOT_POINTER, false>(g, prog.ops[0], pgrid, s);
        if (done) return hipGetLastError();
    }
    bool st = false;
    for (int o = 0; o < prog.nops; ++o) {
        const int op = prog.ops[o].op;
        st |= op == AT_OP_LAP_UPDATE || op == AT_OP_JACOBI || op == AT_OP_DIFFUSE || op == AT_OP_DIFFUSE_ADJ;
    }
    if (g.kind == AT_ROOT_BITMASK) {
        if (st) hipLaunchKernelGGL((k_micro<AT_ROOT_BITMASK, true>), grid, block, 0, s, g, prog);
        else hipLaunchKernelGGL((k_micro<AT_ROOT_BITMASK, false>), grid, block, 0, s, g, prog);
    } else {
        if (st) hipLaunchKernelGGL((k_micro<AT_ROOT_POINTER, true>), grid, block, 0, s, g, prog);
        else hipLaunchKernelGGL((k_micro<AT_ROOT_POINTER, false>), grid, block, 0, s, g, prog);
    }
    return hipGetLastError();
}

// The per-particle part of a particle node: one index-ordered pass
// (k_particles) or, for a gather through the source grid's bins, the gather
// per source bin (k_g2p_bins) and then, when the node has more steps, an
// index-ordered pass for them.
template <int KS, int KD, uint32_t STEPS, int ACT, bool BIN>
static void launch_part_first(const PartProg &pp, dim3 grid, hipStream_t s) {
    if constexpr ((STEPS & PS_G2P) != 0) {
        if (pp.g2p_bins) {
            const int64_t nb = pp.gbin_g.ncells * kG2PSplit < 256 * 8 ? pp.gbin_g.ncells * kG2PSplit : 256 * 8;
            hipLaunchKernelGGL(k_g2p_bins<KS>, dim3((unsigned)nb), dim3(256), 0, s, pp);
            constexpr uint32_t REST = STEPS & ~(uint32_t)PS_G2P;
            if constexpr (REST != 0) hipLaunchKernelGGL((k_particles<KS, KD, REST, ACT, BIN>), grid, dim3(256), 0, s, pp);
            return;
        }
    }
    hipLaunchKernelGGL((k_particles<KS, KD, STEPS, ACT, BIN>), grid, dim3(256), 0, s, pp);
}

// Tiles over bins just made (narrow) or reused (wide).
template <int KD, bool WIDE>
static void launch_p2g_tiles(const PartProg &pp, hipStream_t s) {
    const int64_t nb = pp.gbin_s.ncells < 256 * 8 ? pp.gbin_s.ncells : 256 * 8;
    if (pp.act_mode == AT_ACT_PER_BLOCK)
        hipLaunchKernelGGL((k_p2g_bins<KD, AT_ACT_PER_BLOCK, WIDE>), dim3((unsigned)nb), dim3(256), 0, s, pp);
    else if (pp.act_mode == AT_ACT_NONE)
        hipLaunchKernelGGL((k_p2g_bins<KD, AT_ACT_NONE, WIDE>), dim3((unsigned)nb), dim3(256), 0, s, pp);
    else
        hipLaunchKernelGGL((k_p2g_bins<KD, AT_ACT_PER_NODE, WIDE>), dim3((unsigned)nb), dim3(256), 0, s, pp);
}

template <int KS, int KD, uint32_t STEPS>
static void launch_part_a(const PartProg &pp, dim3 grid, bool bin, hipStream_t s) {
    constexpr bool P2G = (STEPS & PS_P2G) != 0;
    if constexpr ((STEPS & PS_G2P) != 0 && P2G) {
        if (bin && pp.p2g_reuse) {
            // gather through the bins (rewriting their records), advection
            // in particle order, scatter over the same bins
            const int64_t nb = pp.gbin_g.ncells * kG2PSplit < 256 * 8 ? pp.gbin_g.ncells * kG2PSplit : 256 * 8;
            hipLaunchKernelGGL(k_g2p_bins<KS>, dim3((unsigned)nb), dim3(256), 0, s, pp);
            if constexpr ((STEPS & PS_ADVECT) != 0)
                hipLaunchKernelGGL((k_particles<KS, KD, PS_ADVECT, AT_ACT_PER_NODE, false>), grid, dim3(256), 0, s, pp);
            launch_p2g_tiles<KD, true>(pp, s);
            return;
        }
    }
    if (P2G && bin) {
        // cell keys (with the gather and advection), ranks, scan, place, scatter per bin
        if (pp.act_mode == AT_ACT_PER_BLOCK)
            launch_part_first<KS, KD, STEPS, AT_ACT_PER_BLOCK, P2G>(pp, grid, s);
        else if (pp.act_mode == AT_ACT_NONE)
            launch_part_first<KS, KD, STEPS, AT_ACT_NONE, P2G>(pp, grid, s);
        else
            launch_part_first<KS, KD, STEPS, AT_ACT_PER_NODE, P2G>(pp, grid, s);
        if (pp.gdst.ncells <= kHistCells)
            hipLaunchKernelGGL(k_bin_rank<true>, dim3(256), dim3(1024), 0, s, pp.gdst, pp.np);
        else
            hipLaunchKernelGGL(k_bin_rank<false>, dim3(1024), dim3(1024), 0, s, pp.gdst, pp.np);
        hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, pp.gdst);
        hipLaunchKernelGGL(k_bin_place, grid, dim3(256), 0, s, pp);
        launch_p2g_tiles<KD, false>(pp, s);
        return;
    }
    if (pp.act_mode == AT_ACT_PER_BLOCK)
        launch_part_first<KS, KD, STEPS, AT_ACT_PER_BLOCK, false>(pp, grid, s);
    else if (pp.act_mode == AT_ACT_NONE)
        launch_part_first<KS, KD, STEPS, AT_ACT_NONE, false>(pp, grid, s);
    else
        launch_part_first<KS, KD, STEPS, AT_ACT_PER_NODE, false>(pp, grid, s);
}

template <int KS, int KD>
static bool launch_part_s(const PartProg &pp, dim3 grid, bool bin, hipStream_t s) {
    switch (pp.steps) {
    case PS_G2P: launch_part_a<KS, KD, PS_G2P>(pp, grid, bin, s); return true;
    case PS_ADVECT: launch_part_a<KS, KD, PS_ADVECT>(pp, grid, bin, s); return true;
    case PS_P2G: launch_part_a<KS, KD, PS_P2G>(pp, grid, bin, s); return true;
    case PS_G2P | PS_ADVECT: launch_part_a<KS, KD, PS_G2P | PS_ADVECT>(pp, grid, bin, s); return true;
    case PS_ADVECT | PS_P2G: launch_part_a<KS, KD, PS_ADVECT | PS_P2G>(pp, grid, bin, s); return true;
    case PS_G2P | PS_P2G: launch_part_a<KS, KD, PS_G2P | PS_P2G>(pp, grid, bin, s); return true;
    case PS_G2P | PS_ADVECT | PS_P2G: launch_part_a<KS, KD, PS_G2P | PS_ADVECT | PS_P2G>(pp, grid, bin, s); return true;
    default: return false;
    }
}

hipError_t launch_particles(const PartProg &pp, hipStream_t s, int *dispatches) {
    // the scatter is binned when the destination grid has room for every particle
    const bool bin = (pp.steps & PS_P2G) && pp.gdst.pcap >= pp.np;
    const bool split = pp.g2p_bins && (pp.steps & PS_G2P) && (pp.steps & ~(uint32_t)PS_G2P);
    if (bin && pp.p2g_reuse && (pp.steps & PS_G2P))
        *dispatches = (pp.steps & PS_ADVECT) ? 3 : 2;
    else
        *dispatches = (bin ? 5 : 1) + (split ? 1 : 0);
    int64_t blocks = (pp.np + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 256 * 64) blocks = 256 * 64;
    const dim3 grid((unsigned)blocks);
    // a step that does not use a grid takes the other grid's root kind so
    // that only used (kind_src, kind_dst) pairs are instantiated
    const int ks = (pp.steps & PS_G2P) ? pp.gsrc.kind : pp.gdst.kind;
    const int kd = (pp.steps & PS_P2G) ? pp.gdst.kind : ks;
    bool ok;
    if (ks == AT_ROOT_BITMASK && kd == AT_ROOT_BITMASK) ok = launch_part_s<AT_ROOT_BITMASK, AT_ROOT_BITMASK>(pp, grid, bin, s);
    else if (ks == AT_ROOT_BITMASK) ok = launch_part_s<AT_ROOT_BITMASK, AT_ROOT_POINTER>(pp, grid, bin, s);
    else if (kd == AT_ROOT_BITMASK) ok = launch_part_s<AT_ROOT_POINTER, AT_ROOT_BITMASK>(pp, grid, bin, s);
    else ok = launch_part_s<AT_ROOT_POINTER, AT_ROOT_POINTER>(pp, grid, bin, s);
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_scatter_blocks(const GridDev &g, int ch, const int32_t *cells, const float *vals, int64_t n,
                                 hipStream_t s) {
    const unsigned blocks = (unsigned)(n < 65536 ? (n > 0 ? n : 1) : 65536);
    if (g.kind == AT_ROOT_BITMASK)
        hipLaunchKernelGGL(k_scatter_blocks<AT_ROOT_BITMASK>, dim3(blocks), dim3(kSFThreads), 0, s, g, ch, cells, vals, n);
    else
        hipLaunchKernelGGL(k_scatter_blocks<AT_ROOT_POINTER>, dim3(blocks), dim3(kSFThreads), 0, s, g, ch, cells, vals, n);
    return hipGetLastError();
}

hipError_t launch_gather_blocks(const GridDev &g, int ch, const int32_t *cells, float *vals, int64_t n,
                                hipStream_t s) {
    const unsigned blocks = (unsigned)(n < 65536 ? (n > 0 ? n : 1) : 65536);
    if (g.kind == AT_ROOT_BITMASK)
        hipLaunchKernelGGL(k_gather_blocks<AT_ROOT_BITMASK>, dim3(blocks), dim3(kSFThreads), 0, s, g, ch, cells, vals, n);
    else
        hipLaunchKernelGGL(k_gather_blocks<AT_ROOT_POINTER>, dim3(blocks), dim3(kSFThreads), 0, s, g, ch, cells, vals, n);
    return hipGetLastError();
}

template <int KF, int KC>
static void launch_transfer_k(bool restrict_op, const GridDev &f, const GridDev &c, int chf, int chc, float w,
                              bool check, int verify, hipStream_t s) {
    const dim3 grid(wave_grid_size(f, false)), block(64);
    float *xf = f.chan + (int64_t)chf * f.ch_stride;
    float *yc = c.chan + (int64_t)chc * c.ch_stride;
    if (restrict_op) {
        if (check) hipLaunchKernelGGL((k_restrict<KF, KC, true>), grid, block, 0, s, f, c, xf, yc, w, verify);
        else hipLaunchKernelGGL((k_restrict<KF, KC, false>), grid, block, 0, s, f, c, xf, yc, w, verify);
    } else {
        if (check) hipLaunchKernelGGL((k_prolong<KF, KC, true>), grid, block, 0, s, f, c, yc, xf, verify);
        else hipLaunchKernelGGL((k_prolong<KF, KC, false>), grid, block, 0, s, f, c, yc, xf, verify);
    }
}

hipError_t launch_transfer(bool restrict_op, const GridDev &f, const GridDev &c, int chf, int chc, float w,
                           int check, int verify, hipStream_t s) {
    const bool fb = f.kind == AT_ROOT_BITMASK, cb = c.kind == AT_ROOT_BITMASK;
    if (fb && cb) launch_transfer_k<AT_ROOT_BITMASK, AT_ROOT_BITMASK>(restrict_op, f, c, chf, chc, w, check, verify, s);
    else if (fb) launch_transfer_k<AT_ROOT_BITMASK, AT_ROOT_POINTER>(restrict_op, f, c, chf, chc, w, check, verify, s);
    else if (cb) launch_transfer_k<AT_ROOT_POINTER, AT_ROOT_BITMASK>(restrict_op, f, c, chf, chc, w, check, verify, s);
    else launch_transfer_k<AT_ROOT_POINTER, AT_ROOT_POINTER>(restrict_op, f, c, chf, chc, w, check, verify, s);
    return hipGetLastError();
}

hipError_t launch_batch_jacobi(const BatchDev &d, int iters, int workgroups, hipStream_t s) {
    int wgs = workgroups > 0 ? workgroups : 256 * 28;
    wgs = ((wgs + 7) / 8) * 8;
    if (wgs > d.pool) wgs = ((d.pool + 7) / 8) * 8;
    if (wgs < 8) wgs = 8;
    hipLaunchKernelGGL(k_batch_records, dim3(1024), dim3(256), 0, s, d);
    const int W = g_batch_waves;
    for (int it = 0; it < iters; ++it) {
        if (W == 4) {
            hipLaunchKernelGGL((k_batch_lds<4>), dim3(wgs), dim3(256), 0, s, d, it);
            hipLaunchKernelGGL((k_batch<true, 4>), dim3(wgs), dim3(256), 0, s, d, it);
        } else if (W == 2) {
            hipLaunchKernelGGL((k_batch_lds<2>), dim3(wgs), dim3(128), 0, s, d, it);
            hipLaunchKernelGGL((k_batch<true, 2>), dim3(wgs), dim3(128), 0, s, d, it);
        } else {
            hipLaunchKernelGGL((k_batch_lds<1>), dim3(wgs), dim3(64), 0, s, d, it);
            hipLaunchKernelGGL((k_batch<true, 1>), dim3(wgs), dim3(64), 0, s, d, it);
        }
    }
    hipLaunchKernelGGL(k_batch_tick, dim3(1), dim3(64), 0, s, d, iters);
    return hipGetLastError();
}

hipError_t launch_batch_init(const BatchDev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_init, dim3(256), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_batch_retire(const BatchDev &d, const BatchRetireArgs &a, hipStream_t s) {
    if (a.blocks > 0) hipLaunchKernelGGL(k_batch_retire, dim3(a.blocks), dim3(128), 0, s, d, a);
    return hipGetLastError();
}

hipError_t launch_batch_admit(const BatchDev &d, const BatchAdmitArgs &a, hipStream_t s) {
    const int wgs = a.adm_blocks + a.nwork;
    hipLaunchKernelGGL(k_batch_admit, dim3(wgs > 0 ? wgs : 1), dim3(128), 0, s, d, a);
    return hipGetLastError();
}

hipError_t launch_popcount(const GridDev &g, hipStream_t s) {
    hipLaunchKernelGGL(k_popcount, dim3(1), dim3(1024), 0, s, g);
    return hipGetLastError();
}

// ------------------------------------------------- static binning workspace
// The binning workspace of a scatter that must not allocate: one file-scope
// device array, which every device that loads this library holds for the
// life of the process.  Segments, each 256-byte aligned: per-cell counts,
// first positions and bins (kStaticCells each), per-particle keys, records
// and outlier indices (kStaticParticles each).
constexpr size_t kStaticSegCount = 0;
constexpr size_t kStaticSegOff = kStaticSegCount + (size_t)kStaticCells * sizeof(int32_t);
constexpr size_t kStaticSegBins = kStaticSegOff + (size_t)kStaticCells * sizeof(int32_t);
constexpr size_t kStaticSegKr = kStaticSegBins + (size_t)kStaticCells * sizeof(int4);
constexpr size_t kStaticSegStage = kStaticSegKr + (size_t)kStaticParticles * sizeof(int2);
constexpr size_t kStaticSegOut = kStaticSegStage + 2 * (size_t)kStaticParticles * sizeof(float4);
constexpr size_t kStaticBytes = kStaticSegOut + (size_t)kStaticParticles * sizeof(int32_t);
static_assert(kStaticSegOff % 256 == 0 && kStaticSegBins % 256 == 0 && kStaticSegKr % 256 == 0 &&
              kStaticSegStage % 256 == 0 && kStaticSegOut % 256 == 0, "segments must stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device
}  // namespace

size_t static_workspace_bytes() { return kStaticBytes; }

hipError_t static_bin_workspace(GridDev &g, int64_t np, hipStream_t s) {
    if (np < 0 || np > kStaticParticles || g.ncells > kStaticCells) return hipErrorInvalidValue;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            // the array's own name is a host-side stand-in: its device
            // address comes from the runtime, once per device
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            if (!p) return hipErrorInvalidSymbol;
            g_scratch_ptr[dev] = (unsigned char *)p;
        }
        base = g_scratch_ptr[dev];
    }
    g.pcap = kStaticParticles;
    g.pcount = (int32_t *)(base + kStaticSegCount);
    g.poff = (int32_t *)(base + kStaticSegOff);
    g.pbins = (int4 *)(base + kStaticSegBins);
    g.pkr = (int2 *)(base + kStaticSegKr);
    g.pstage = (float4 *)(base + kStaticSegStage);
    g.pout = (int32_t *)(base + kStaticSegOut);
    int64_t blocks = (g.ncells + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_static_clear, dim3((unsigned)blocks), dim3(256), 0, s, g.pcount, g.ncells, g.hdr);
    return hipGetLastError();
}

}  // namespace ats
