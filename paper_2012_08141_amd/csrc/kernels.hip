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

#include "internal.hpp"

namespace ats {
namespace {

constexpr int kSFThreads = 128;          // struct-for workgroup
constexpr int kTile = 1600;              // 10 x 10 x 16 floats (k padded to 16)
constexpr int kSpinLimit = 1 << 22;      // bounded wait on a pointer-root allocation
int g_sf_grid_override = 0;

// -------------------------------------------------------------- root access

__device__ __forceinline__ bool bit_set(const uint32_t *bits, int64_t c) {
    return (bits[c >> 5] >> (c & 31)) & 1u;
}

// Slot of root cell c, or -1 when the block is inactive (no concurrent
// activation of the same grid may be running).
template <int KIND>
__device__ __forceinline__ int32_t slot_of(const GridDev &g, int64_t c) {
    if (KIND == AT_ROOT_BITMASK) return bit_set(g.bits, c) ? (int32_t)c : -1;
    const int32_t s = g.ptr[c];
    return s >= 0 ? s : -1;
}

// Activation on write: make root cell c active and return its slot (-1 if a
// pointer pool is exhausted).  Inactive leaf storage is kept at zero (the
// grid starts zeroed and leaves only become inactive through a clear that
// zeroes them), so a newly activated block reads 0 without a fill here.
//
// Pointer root: the first thread to CAS the cell from NULL to LOCKED takes a
// slot from the bump counter and publishes it; the others wait for the
// publication.  The publish sits in an if-block that every lane of the wave
// finishes before any lane reaches the wait loop after it, so a waiting lane
// never blocks the lane it waits for.  The wait is bounded.
template <int KIND>
__device__ __forceinline__ int32_t activate_cell(const GridDev &g, int64_t c) {
    const uint32_t m = 1u << (c & 31);
    if (KIND == AT_ROOT_BITMASK) {
        const uint32_t w = __hip_atomic_load(&g.bits[c >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!(w & m)) atomicOr(&g.bits[c >> 5], m);
        return (int32_t)c;
    }
    int32_t s = __hip_atomic_load(&g.ptr[c], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (s == PTR_NULL) {
        const int32_t old = atomicCAS(&g.ptr[c], PTR_NULL, PTR_LOCKED);
        if (old == PTR_NULL) {
            int32_t ns = atomicAdd(&g.hdr[HDR_BUMP], 1);
            if (ns >= g.cap) {
                atomicOr(&g.hdr[HDR_ERR], ERR_CAPACITY);
                ns = PTR_FAILED;
            } else {
                atomicOr(&g.bits[c >> 5], m);
            }
            __hip_atomic_store(&g.ptr[c], ns, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            s = ns;
        } else {
            s = old;
        }
    }
    for (int it = 0; s == PTR_LOCKED; ++it) {
        if (it >= kSpinLimit) {
            atomicOr(&g.hdr[HDR_ERR], ERR_SPIN);
            s = PTR_FAILED;
            break;
        }
        __builtin_amdgcn_s_sleep(2);
        s = __hip_atomic_load(&g.ptr[c], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    }
    return s >= 0 ? s : -1;
}

__device__ __forceinline__ float *chan(const GridDev &g, int c) { return g.chan + (int64_t)c * g.ch_stride; }

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

__device__ __forceinline__ void cell_coords(const GridDev &g, int32_t cell, int &bi, int &bj, int &bk) {
    bi = cell / g.R2;
    const int r = cell - bi * g.R2;
    bj = r / g.R;
    bk = r - bj * g.R;
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
// One workgroup of 1024 threads.  Thread t owns a contiguous run of mask
// words; a block-wide exclusive scan of per-thread popcounts gives every
// thread its output offset, so the list comes out in ascending cell order
// with no atomics.  The count is written by the last thread (the clear of
// the previous list is folded in: the count is simply overwritten).
__global__ __launch_bounds__(1024) void k_listgen(GridDev g) {
    __shared__ int wsum[16];
    const int64_t W = (g.ncells + 31) >> 5;
    const int tid = threadIdx.x;
    const int T = blockDim.x;
    const int64_t per = (W + T - 1) / T;
    const int64_t w0 = min((int64_t)tid * per, W);
    const int64_t w1 = min(w0 + per, W);
    const uint32_t tail = (g.ncells & 31) ? ((1u << (g.ncells & 31)) - 1u) : 0xffffffffu;
    int cnt = 0;
    for (int64_t w = w0; w < w1; ++w) {
        uint32_t b = g.bits[w];
        if (w == W - 1) b &= tail;
        cnt += __popc(b);
    }
    const int incl = wave_incl_scan(cnt);
    const int lane = tid & 63, wid = tid >> 6, nw = (T + 63) >> 6;
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        const int v = lane < nw ? wsum[lane] : 0;
        const int iv = wave_incl_scan(v);
        if (lane < nw) wsum[lane] = iv - v;
    }
    __syncthreads();
    int pos = wsum[wid] + incl - cnt;
    for (int64_t w = w0; w < w1; ++w) {
        uint32_t b = g.bits[w];
        if (w == W - 1) b &= tail;
        while (b) {
            const int bit = __builtin_ctz(b);
            g.list[pos++] = (int32_t)(w * 32 + bit);
            b &= b - 1;
        }
    }
    if (tid == T - 1) g.hdr[HDR_COUNT] = pos;
}

// ----------------------------------------------------- 7-point stencils (LDS)
// The block plus a one-voxel face halo is staged in an LDS tile of
// 10 x 10 x 16 floats per stencil-read channel: plane stride 160, row stride
// 16, local k at column k + 4 so every interior row is two aligned float4s.
// Halo faces come from the six face-neighbour blocks (zeros when inactive or
// outside the domain): i and j faces as float4 rows, k faces as scalars.

struct StencilCh {
    const float *tin[3];  // stencil-read channels (tile order)
    const float *ein;     // elementwise input (JACOBI: b; DIFFUSE_ADJ: gk)
    float *out0;          // output (LAP/DIFFUSE: out; JACOBI: xn; ADJ: lam)
    float *out1;          // DIFFUSE_ADJ: gk
};

template <int OP> struct NTiles { static constexpr int v = 1; };
template <> struct NTiles<AT_OP_DIFFUSE> { static constexpr int v = 2; };
template <> struct NTiles<AT_OP_DIFFUSE_ADJ> { static constexpr int v = 3; };

// Values around the thread's four voxels: c[q] centre, f[face][q] the
// neighbour across `face` (order i-1, i+1, j-1, j+1, k-1, k+1).
struct Around {
    float c[4];
    float f[6][4];
};

__device__ __forceinline__ void gather_around(const float *tile, int rb, Around &a) {
    const float4 C = *reinterpret_cast<const float4 *>(tile + rb);
    const float4 IM = *reinterpret_cast<const float4 *>(tile + rb - 160);
    const float4 IP = *reinterpret_cast<const float4 *>(tile + rb + 160);
    const float4 JM = *reinterpret_cast<const float4 *>(tile + rb - 16);
    const float4 JP = *reinterpret_cast<const float4 *>(tile + rb + 16);
    const float KL = tile[rb - 1];
    const float KR = tile[rb + 4];
    a.c[0] = C.x; a.c[1] = C.y; a.c[2] = C.z; a.c[3] = C.w;
    a.f[0][0] = IM.x; a.f[0][1] = IM.y; a.f[0][2] = IM.z; a.f[0][3] = IM.w;
    a.f[1][0] = IP.x; a.f[1][1] = IP.y; a.f[1][2] = IP.z; a.f[1][3] = IP.w;
    a.f[2][0] = JM.x; a.f[2][1] = JM.y; a.f[2][2] = JM.z; a.f[2][3] = JM.w;
    a.f[3][0] = JP.x; a.f[3][1] = JP.y; a.f[3][2] = JP.z; a.f[3][3] = JP.w;
    a.f[4][0] = KL;   a.f[4][1] = C.x;  a.f[4][2] = C.y;  a.f[4][3] = C.z;
    a.f[5][0] = C.y;  a.f[5][1] = C.z;  a.f[5][2] = C.w;  a.f[5][3] = KR;
}

__device__ __forceinline__ float nbsum(const Around &a, int q) {
    float s = a.f[0][q] + a.f[1][q];
    s = s + a.f[2][q];
    s = s + a.f[3][q];
    s = s + a.f[4][q];
    s = s + a.f[5][q];
    return s;
}

template <int OP, int KIND, bool CHECK>
__global__ __launch_bounds__(kSFThreads) void k_stencil(GridDev g, StencilCh c, float p) {
    constexpr int NT = NTiles<OP>::v;
    __shared__ float4 tile4[NT * kTile / 4];
    float *tile = reinterpret_cast<float *>(tile4);
    const int t = threadIdx.x;
    const int li = t >> 4, lj = (t >> 1) & 7, k0 = (t & 1) * 4;
    const int rb = (li + 1) * 160 + (lj + 1) * 16 + 4 + k0;
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int32_t cell = g.list[e];
        int bi, bj, bk;
        cell_coords(g, cell, bi, bj, bk);
        const int32_t slot = (KIND == AT_ROOT_BITMASK) ? cell : g.ptr[cell];
        __syncthreads();   // the previous block's tile reads are done
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const float4 v = reinterpret_cast<const float4 *>(c.tin[nt] + (int64_t)slot * kBV)[t];
            *reinterpret_cast<float4 *>(tile + nt * kTile + rb) = v;
        }
        if (t < 64) {
            const int face = t >> 4, q = t & 15, a = q >> 1, kk = (q & 1) * 4;
            int64_t nc = -1;
            int src, dst;
            if (face == 0) {        // i-1: neighbour's i = 7 plane, row j = a
                if (bi > 0) nc = cell - g.R2;
                src = 7 * 64 + a * 8 + kk; dst = 0 * 160 + (a + 1) * 16 + 4 + kk;
            } else if (face == 1) { // i+1: neighbour's i = 0 plane
                if (bi < g.R - 1) nc = cell + g.R2;
                src = 0 * 64 + a * 8 + kk; dst = 9 * 160 + (a + 1) * 16 + 4 + kk;
            } else if (face == 2) { // j-1: neighbour's j = 7 rows, plane i = a
                if (bj > 0) nc = cell - g.R;
                src = a * 64 + 7 * 8 + kk; dst = (a + 1) * 160 + 0 * 16 + 4 + kk;
            } else {                // j+1
                if (bj < g.R - 1) nc = cell + g.R;
                src = a * 64 + 0 * 8 + kk; dst = (a + 1) * 160 + 9 * 16 + 4 + kk;
            }
            const int32_t ns = nc >= 0 ? slot_of<KIND>(g, nc) : -1;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (ns >= 0) v = *reinterpret_cast<const float4 *>(c.tin[nt] + (int64_t)ns * kBV + src);
                *reinterpret_cast<float4 *>(tile + nt * kTile + dst) = v;
            }
        } else {
            const int q = t - 64, a = q >> 3, b = q & 7;
            const int32_t sm = bk > 0 ? slot_of<KIND>(g, cell - 1) : -1;
            const int32_t sp = bk < g.R - 1 ? slot_of<KIND>(g, cell + 1) : -1;
            const int row = (a + 1) * 160 + (b + 1) * 16;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                tile[nt * kTile + row + 3] = sm >= 0 ? c.tin[nt][(int64_t)sm * kBV + a * 64 + b * 8 + 7] : 0.f;
                tile[nt * kTile + row + 12] = sp >= 0 ? c.tin[nt][(int64_t)sp * kBV + a * 64 + b * 8 + 0] : 0.f;
            }
        }
        __syncthreads();
        int32_t wslot = slot;
        if (CHECK) wslot = activate_cell<KIND>(g, cell);
        const int64_t off = (int64_t)wslot * kBV + 4 * t;
        if (OP == AT_OP_LAP_UPDATE) {
            Around A;
            gather_around(tile, rb, A);
            float r[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float s = nbsum(A, q);
                const float six_a = 6.0f * A.c[q];
                const float d = s - six_a;
                const float tq = p * d;
                r[q] = A.c[q] + tq;
            }
            *reinterpret_cast<float4 *>(c.out0 + off) = make_float4(r[0], r[1], r[2], r[3]);
        } else if (OP == AT_OP_JACOBI) {
            Around X;
            gather_around(tile, rb, X);
            const float4 b = *reinterpret_cast<const float4 *>(c.ein + (int64_t)slot * kBV + 4 * t);
            const float bb[4] = {b.x, b.y, b.z, b.w};
            const float sixth = 0x1.555556p-3f;
            float r[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float s = nbsum(X, q);
                const float tq = s + bb[q];
                r[q] = tq * sixth;
            }
            *reinterpret_cast<float4 *>(c.out0 + off) = make_float4(r[0], r[1], r[2], r[3]);
        } else if (OP == AT_OP_DIFFUSE) {
            Around A, K;
            gather_around(tile, rb, A);
            gather_around(tile + kTile, rb, K);
            float r[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float f = 0.f;
#pragma unroll
                for (int fc = 0; fc < 6; ++fc) {
                    const float kf = 0.5f * (K.c[q] + K.f[fc][q]);
                    f = f + kf * (A.f[fc][q] - A.c[q]);
                }
                r[q] = A.c[q] + p * f;
            }
            *reinterpret_cast<float4 *>(c.out0 + off) = make_float4(r[0], r[1], r[2], r[3]);
        } else if (OP == AT_OP_DIFFUSE_ADJ) {
            Around A, K, L;
            gather_around(tile, rb, A);
            gather_around(tile + kTile, rb, K);
            gather_around(tile + 2 * kTile, rb, L);
            const float4 gk4 = *reinterpret_cast<const float4 *>(c.ein + (int64_t)slot * kBV + 4 * t);
            const float gk[4] = {gk4.x, gk4.y, gk4.z, gk4.w};
            const float half_dt = p * 0.5f;
            float rl[4], rg[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float f = 0.f, q2 = 0.f;
#pragma unroll
                for (int fc = 0; fc < 6; ++fc) {
                    const float kf = 0.5f * (K.c[q] + K.f[fc][q]);
                    f = f + kf * (L.f[fc][q] - L.c[q]);
                    q2 = q2 + (A.f[fc][q] - A.c[q]) * (L.c[q] - L.f[fc][q]);
                }
                rl[q] = L.c[q] + p * f;
                rg[q] = gk[q] + half_dt * q2;
            }
            *reinterpret_cast<float4 *>(c.out0 + off) = make_float4(rl[0], rl[1], rl[2], rl[3]);
            *reinterpret_cast<float4 *>(c.out1 + off) = make_float4(rg[0], rg[1], rg[2], rg[3]);
        }
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

template <int KIND>
__global__ __launch_bounds__(kSFThreads) void k_micro(GridDev g, MicroProg prog) {
    const int t = threadIdx.x;
    const int li = t >> 4, lj = (t >> 1) & 7, k0 = (t & 1) * 4;
    bool has_stencil = false;
    for (int o = 0; o < prog.nops; ++o) {
        const int op = prog.ops[o].op;
        has_stencil |= (op == AT_OP_LAP_UPDATE || op == AT_OP_JACOBI || op == AT_OP_DIFFUSE || op == AT_OP_DIFFUSE_ADJ);
    }
    const ListRange lr = list_range(g.hdr[HDR_COUNT]);
    for (int e = lr.lo; e < lr.hi; e += lr.step) {
        const int32_t cell = g.list[e];
        int32_t slot = (KIND == AT_ROOT_BITMASK) ? cell : g.ptr[cell];
        int32_t nbs[6] = {-1, -1, -1, -1, -1, -1};
        if (has_stencil) {
            int bi, bj, bk;
            cell_coords(g, cell, bi, bj, bk);
            if (bi > 0) nbs[0] = slot_of<KIND>(g, cell - g.R2);
            if (bi < g.R - 1) nbs[1] = slot_of<KIND>(g, cell + g.R2);
            if (bj > 0) nbs[2] = slot_of<KIND>(g, cell - g.R);
            if (bj < g.R - 1) nbs[3] = slot_of<KIND>(g, cell + g.R);
            if (bk > 0) nbs[4] = slot_of<KIND>(g, cell - 1);
            if (bk < g.R - 1) nbs[5] = slot_of<KIND>(g, cell + 1);
        }
        if (prog.check) slot = activate_cell<KIND>(g, cell);
        const int64_t off = (int64_t)slot * kBV + 4 * t;
        for (int o = 0; o < prog.nops; ++o) {
            const MicroOp &op = prog.ops[o];
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
            case AT_OP_LAP_UPDATE:
            case AT_OP_JACOBI:
            case AT_OP_DIFFUSE:
            case AT_OP_DIFFUSE_ADJ: {
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

template <int KS, int KD, uint32_t STEPS, int ACT>
__global__ __launch_bounds__(256) void k_particles(PartProg pp) {
    const int64_t np = pp.np;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        float x[3] = {pp.x[p], pp.x[np + p], pp.x[2 * np + p]};
        float v[3];
        if (STEPS & PS_G2P) {
            const GridDev &g = pp.gsrc;
            const int N = g.R * kBS;
            float w[3][3];
            int base[3];
            for (int c = 0; c < 3; ++c) base[c] = bspline(x[c] * pp.inv_dx_src, w[c]);
            const float *V0 = chan(g, pp.ch_vsrc), *V1 = chan(g, pp.ch_vsrc + 1), *V2 = chan(g, pp.ch_vsrc + 2);
            float acc[3] = {0.f, 0.f, 0.f};
            for (int a = 0; a < 3; ++a) {
                const int i = base[0] + a;
                for (int b = 0; b < 3; ++b) {
                    const int j = base[1] + b;
                    const float wab = w[0][a] * w[1][b];
                    for (int d = 0; d < 3; ++d) {
                        const int k = base[2] + d;
                        const float wt = wab * w[2][d];
                        float n0 = 0.f, n1 = 0.f, n2 = 0.f;
                        if (i >= 0 && j >= 0 && k >= 0 && i < N && j < N && k < N) {
                            const int64_t cell = ((int64_t)(i >> 3) * g.R + (j >> 3)) * g.R + (k >> 3);
                            const int32_t s = slot_of<KS>(g, cell);
                            if (s >= 0) {
                                const int64_t o = (int64_t)s * kBV + (i & 7) * 64 + (j & 7) * 8 + (k & 7);
                                n0 = V0[o]; n1 = V1[o]; n2 = V2[o];
                            }
                        }
                        acc[0] = acc[0] + wt * n0;
                        acc[1] = acc[1] + wt * n1;
                        acc[2] = acc[2] + wt * n2;
                    }
                }
            }
            v[0] = acc[0]; v[1] = acc[1]; v[2] = acc[2];
            pp.v[p] = v[0]; pp.v[np + p] = v[1]; pp.v[2 * np + p] = v[2];
        } else {
            v[0] = pp.v[p]; v[1] = pp.v[np + p]; v[2] = pp.v[2 * np + p];
        }
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
            const float mp = pp.m[p];
            float *M = chan(g, pp.ch_m), *MV0 = chan(g, pp.ch_mv), *MV1 = chan(g, pp.ch_mv + 1),
                  *MV2 = chan(g, pp.ch_mv + 2);
            // per-block activation: the touched nodes span at most 2 blocks per axis
            int32_t bslot[2][2][2];
            const int blo[3] = {base[0] >> 3, base[1] >> 3, base[2] >> 3};
            if (ACT == AT_ACT_PER_BLOCK) {
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int d = 0; d < 2; ++d) {
                            const int ci = blo[0] + a, cj = blo[1] + b, ck = blo[2] + d;
                            bslot[a][b][d] = -1;
                            const bool used = (a == 0 || ((base[0] + 2) >> 3) != blo[0]) &&
                                              (b == 0 || ((base[1] + 2) >> 3) != blo[1]) &&
                                              (d == 0 || ((base[2] + 2) >> 3) != blo[2]);
                            if (!used || ci < 0 || cj < 0 || ck < 0 || ci >= g.R || cj >= g.R || ck >= g.R) continue;
                            bslot[a][b][d] = activate_cell<KD>(g, ((int64_t)ci * g.R + cj) * g.R + ck);
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
                        if (ACT == AT_ACT_PER_BLOCK) {
                            s = bslot[(i >> 3) - blo[0]][(j >> 3) - blo[1]][(k >> 3) - blo[2]];
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

void set_struct_for_grid_size(int wgs) { g_sf_grid_override = wgs > 0 ? ((wgs + 7) / 8) * 8 : 0; }

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

hipError_t launch_listgen(const GridDev &g, hipStream_t s) {
    hipLaunchKernelGGL(k_listgen, dim3(1), dim3(1024), 0, s, g);
    return hipGetLastError();
}

template <int OP, int KIND>
static void launch_stencil_t(const GridDev &g, const StencilCh &c, float p, int check, hipStream_t s) {
    const dim3 grid(struct_for_grid_size(g)), block(kSFThreads);
    if (check)
        hipLaunchKernelGGL((k_stencil<OP, KIND, true>), grid, block, 0, s, g, c, p);
    else
        hipLaunchKernelGGL((k_stencil<OP, KIND, false>), grid, block, 0, s, g, c, p);
}

template <int OP>
static void launch_stencil_k(const GridDev &g, const StencilCh &c, float p, int check, hipStream_t s) {
    if (g.kind == AT_ROOT_BITMASK) launch_stencil_t<OP, AT_ROOT_BITMASK>(g, c, p, check, s);
    else launch_stencil_t<OP, AT_ROOT_POINTER>(g, c, p, check, s);
}

hipError_t launch_stencil(const GridDev &g, int op, const int32_t *ch, float p, int check, hipStream_t s) {
    StencilCh c{};
    auto C = [&](int i) { return g.chan + (int64_t)ch[i] * g.ch_stride; };
    switch (op) {
    case AT_OP_LAP_UPDATE:
        c.tin[0] = C(0); c.out0 = C(1);
        launch_stencil_k<AT_OP_LAP_UPDATE>(g, c, p, check, s);
        break;
    case AT_OP_JACOBI:
        c.tin[0] = C(0); c.ein = C(1); c.out0 = C(2);
        launch_stencil_k<AT_OP_JACOBI>(g, c, p, check, s);
        break;
    case AT_OP_DIFFUSE:
        c.tin[0] = C(0); c.tin[1] = C(1); c.out0 = C(2);
        launch_stencil_k<AT_OP_DIFFUSE>(g, c, p, check, s);
        break;
    case AT_OP_DIFFUSE_ADJ:
        c.tin[0] = C(0); c.tin[1] = C(1); c.tin[2] = C(2); c.out0 = C(3); c.ein = C(4); c.out1 = C(4);
        launch_stencil_k<AT_OP_DIFFUSE_ADJ>(g, c, p, check, s);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_micro(const GridDev &g, const MicroProg &prog, hipStream_t s) {
    const dim3 grid(struct_for_grid_size(g)), block(kSFThreads);
    if (g.kind == AT_ROOT_BITMASK)
        hipLaunchKernelGGL(k_micro<AT_ROOT_BITMASK>, grid, block, 0, s, g, prog);
    else
        hipLaunchKernelGGL(k_micro<AT_ROOT_POINTER>, grid, block, 0, s, g, prog);
    return hipGetLastError();
}

template <int KS, int KD, uint32_t STEPS>
static void launch_part_a(const PartProg &pp, dim3 grid, hipStream_t s) {
    if (pp.act_mode == AT_ACT_PER_BLOCK)
        hipLaunchKernelGGL((k_particles<KS, KD, STEPS, AT_ACT_PER_BLOCK>), grid, dim3(256), 0, s, pp);
    else
        hipLaunchKernelGGL((k_particles<KS, KD, STEPS, AT_ACT_PER_NODE>), grid, dim3(256), 0, s, pp);
}

template <int KS, int KD>
static bool launch_part_s(const PartProg &pp, dim3 grid, hipStream_t s) {
    switch (pp.steps) {
    case PS_G2P: launch_part_a<KS, KD, PS_G2P>(pp, grid, s); return true;
    case PS_ADVECT: launch_part_a<KS, KD, PS_ADVECT>(pp, grid, s); return true;
    case PS_P2G: launch_part_a<KS, KD, PS_P2G>(pp, grid, s); return true;
    case PS_G2P | PS_ADVECT: launch_part_a<KS, KD, PS_G2P | PS_ADVECT>(pp, grid, s); return true;
    case PS_ADVECT | PS_P2G: launch_part_a<KS, KD, PS_ADVECT | PS_P2G>(pp, grid, s); return true;
    case PS_G2P | PS_P2G: launch_part_a<KS, KD, PS_G2P | PS_P2G>(pp, grid, s); return true;
    case PS_G2P | PS_ADVECT | PS_P2G: launch_part_a<KS, KD, PS_G2P | PS_ADVECT | PS_P2G>(pp, grid, s); return true;
    default: return false;
    }
}

hipError_t launch_particles(const PartProg &pp, hipStream_t s) {
    int64_t blocks = (pp.np + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 256 * 64) blocks = 256 * 64;
    const dim3 grid((unsigned)blocks);
    // a step that does not use a grid takes the other grid's root kind so
    // that only used (kind_src, kind_dst) pairs are instantiated
    const int ks = (pp.steps & PS_G2P) ? pp.gsrc.kind : pp.gdst.kind;
    const int kd = (pp.steps & PS_P2G) ? pp.gdst.kind : ks;
    bool ok;
    if (ks == AT_ROOT_BITMASK && kd == AT_ROOT_BITMASK) ok = launch_part_s<AT_ROOT_BITMASK, AT_ROOT_BITMASK>(pp, grid, s);
    else if (ks == AT_ROOT_BITMASK) ok = launch_part_s<AT_ROOT_BITMASK, AT_ROOT_POINTER>(pp, grid, s);
    else if (kd == AT_ROOT_BITMASK) ok = launch_part_s<AT_ROOT_POINTER, AT_ROOT_BITMASK>(pp, grid, s);
    else ok = launch_part_s<AT_ROOT_POINTER, AT_ROOT_POINTER>(pp, grid, s);
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

hipError_t launch_popcount(const GridDev &g, hipStream_t s) {
    hipLaunchKernelGGL(k_popcount, dim3(1), dim3(1024), 0, s, g);
    return hipGetLastError();
}

}  // namespace ats
