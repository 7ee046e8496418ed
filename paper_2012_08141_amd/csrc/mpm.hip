// MLS-MPM particle kernels for gfx950 (the falling cube of the paper's
// Section 8.3): the gather with the APIC affine matrix (G2P), advection, and
// the scatter with the fixed-corotated stress (P2G), alone or fused into one
// G2P2G pass in which the gathered v and C and the advected x reach the
// scatter in registers.
//
// One workgroup of 256 threads takes a chunk of 256 consecutive particles
// (one per thread).  The chunk's nodes -- the bounding box of the 27-node
// neighbourhoods of its particles -- form a tile held in LDS when it has at
// most kTileMax nodes and spans at most kTileBlocks leaf blocks:
//   * the gather first loads the tile of the three velocity channels with
//     one root lookup per leaf block, then every particle gathers from LDS;
//   * the scatter sorts the chunk's particles by base node (a counting sort
//     with integer LDS atomics) into LDS records.  One work item per (base
//     node, offset) sums the four channels' contributions of that base's
//     particles to the node at that offset and stages them in LDS (each
//     staged sum has one writer); then one thread per tile node adds up the
//     at most 27 staged sums landing on its node, offsets in (a, b, d)
//     order, and adds the four totals to the grid with one global atomic
//     each.  Work items of one base sit in neighbouring lanes, so they run
//     the same number of particles and read the same records (LDS
//     broadcast).  No LDS float atomic is used: measured, they are an order
//     of magnitude too slow here.  The touched blocks are activated once per
//     workgroup.
// Spatially ordered particle arrays make compact tiles; a chunk whose box is
// too large falls back to per-node root lookups and global atomics, with the
// same result.  Chunks are dealt to the 8 XCDs in contiguous ranges, so
// neighbouring chunks (whose tiles overlap) share an L2.
//
// Nothing here is a dense contraction: no MFMA.  The arithmetic of one
// particle follows the order documented in include/atsparse.h
// (at_p2g_mls, at_g2p_apic), without contraction.
#include <hip/hip_runtime.h>

#include <climits>

#include "internal.hpp"

namespace ats {
namespace {

#include "grid_device.hpp"

constexpr int kMT = 256;          // particles per chunk, threads per workgroup
constexpr int kTileMax = 512;     // nodes of an LDS tile
constexpr int kMaxKeys = 96;      // base nodes a chunk's scatter may have for the tiled path
constexpr int kRec = 15;          // floats per particle record of the scatter
constexpr int kTileBlocks = 64;   // leaf blocks a tile may span
constexpr int kPolarIters = 16;   // bound on the Newton iterations of the polar decomposition

__device__ __forceinline__ int32_t lookup(const GridDev &g, int64_t cell) {
    return g.kind == AT_ROOT_BITMASK ? slot_of<AT_ROOT_BITMASK>(g, cell) : slot_of<AT_ROOT_POINTER>(g, cell);
}

__device__ __forceinline__ int32_t activate(const GridDev &g, int64_t cell) {
    return g.kind == AT_ROOT_BITMASK ? activate_cell<AT_ROOT_BITMASK>(g, cell) : activate_cell<AT_ROOT_POINTER>(g, cell);
}

__device__ __forceinline__ bool in_domain(int i, int j, int k, int n) {
    return i >= 0 && j >= 0 && k >= 0 && i < n && j < n && k < n;
}

// Quadratic B-spline of one axis: base = floor(X - 1/2), fx = X - base.
__device__ __forceinline__ int spline(float X, float w[3], float &fx) {
    const int base = (int)floorf(X - 0.5f);
    fx = X - (float)base;
    const float t0 = 1.5f - fx, t1 = fx - 1.0f, t2 = fx - 0.5f;
    w[0] = 0.5f * (t0 * t0);
    w[1] = 0.75f - t1 * t1;
    w[2] = 0.5f * (t2 * t2);
    return base;
}

__device__ __forceinline__ float det3(const float *A) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// Rotation of the polar decomposition F = R S by Newton's iteration
// R <- (R + R^-T) / 2 from R = F (R^-T = cofactor matrix / det), until no
// entry moves by more than 1e-6 (at most kPolarIters iterations).
__device__ __forceinline__ void polar_rotation(const float F[9], float R[9]) {
#pragma unroll
    for (int q = 0; q < 9; ++q) R[q] = F[q];
    for (int it = 0; it < kPolarIters; ++it) {
        const float d = det3(R);
        const float inv = 1.0f / d;
        float cof[9];
        cof[0] = R[4] * R[8] - R[5] * R[7];
        cof[1] = R[5] * R[6] - R[3] * R[8];
        cof[2] = R[3] * R[7] - R[4] * R[6];
        cof[3] = R[2] * R[7] - R[1] * R[8];
        cof[4] = R[0] * R[8] - R[2] * R[6];
        cof[5] = R[1] * R[6] - R[0] * R[7];
        cof[6] = R[1] * R[5] - R[2] * R[4];
        cof[7] = R[2] * R[3] - R[0] * R[5];
        cof[8] = R[0] * R[4] - R[1] * R[3];
        float moved = 0.0f;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const float nx = 0.5f * (R[q] + cof[q] * inv);
            moved = fmaxf(moved, fabsf(nx - R[q]));
            R[q] = nx;
        }
        if (moved <= 1e-6f) break;
    }
}

// The chunk's tile: nodes [lo, lo + ext) per axis, leaf blocks
// [blo, blo + bext) per axis.
struct Tile {
    int lo[3], ext[3], blo[3], bext[3];
    int nodes, blocks;
    bool fits;
};

// Bounding box of base .. base + 2 over the workgroup's valid lanes.
__device__ __forceinline__ Tile tile_of(const int base[3], bool valid, int *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int mn[3], mx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        mn[c] = valid ? base[c] : INT_MAX;
        mx[c] = valid ? base[c] : INT_MIN;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            mn[c] = min(mn[c], __shfl_xor(mn[c], o, 64));
            mx[c] = max(mx[c], __shfl_xor(mx[c], o, 64));
        }
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            red[c * 4 + wid] = mn[c];
            red[12 + c * 4 + wid] = mx[c];
        }
    __syncthreads();
    Tile T;
    int64_t nodes = 1, blocks = 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int lo = red[c * 4], hi = red[12 + c * 4];
        for (int w = 1; w < kMT / 64; ++w) {
            lo = min(lo, red[c * 4 + w]);
            hi = max(hi, red[12 + c * 4 + w]);
        }
        const int64_t ext = (int64_t)hi - lo + 3;
        T.lo[c] = lo;
        T.ext[c] = ext < INT_MAX ? (int)ext : INT_MAX;
        T.blo[c] = lo >> 3;                                     // floor for negative nodes too
        const int64_t bext = (((int64_t)lo + ext - 1) >> 3) - T.blo[c] + 1;
        T.bext[c] = bext < INT_MAX ? (int)bext : INT_MAX;
        nodes *= ext;
        blocks *= bext;
        if (nodes > kTileMax) nodes = kTileMax + 1;
        if (blocks > kTileBlocks) blocks = kTileBlocks + 1;
    }
    T.nodes = (int)nodes;
    T.blocks = (int)blocks;
    T.fits = nodes <= kTileMax && blocks <= kTileBlocks &&
             (int64_t)(T.ext[0] - 2) * (T.ext[1] - 2) * (T.ext[2] - 2) <= kMaxKeys;
    __syncthreads();   // red is reused by the next call
    return T;
}

// Tile block index of node (i, j, k) (inside the tile).
__device__ __forceinline__ int tile_block(const Tile &T, int i, int j, int k) {
    return (((i >> 3) - T.blo[0]) * T.bext[1] + ((j >> 3) - T.blo[1])) * T.bext[2] + ((k >> 3) - T.blo[2]);
}

__device__ __forceinline__ int64_t block_cell(const GridDev &g, const Tile &T, int b) {
    const int bk = b % T.bext[2], bj = (b / T.bext[2]) % T.bext[1], bi = b / (T.bext[1] * T.bext[2]);
    const int gi = T.blo[0] + bi, gj = T.blo[1] + bj, gk = T.blo[2] + bk;
    if (gi < 0 || gj < 0 || gk < 0 || gi >= g.R || gj >= g.R || gk >= g.R) return -1;
    return ((int64_t)gi * g.R + gj) * g.R + gk;
}

__device__ __forceinline__ int64_t voxel_offset(int i, int j, int k) { return (i & 7) * 64 + (j & 7) * 8 + (k & 7); }

struct Chunks {
    int64_t first, end, step;
};
// Chunks of this workgroup: each XCD (workgroups are dealt to the 8 XCDs
// round-robin) walks one contiguous eighth of the chunk range.
__device__ __forceinline__ Chunks chunks_of(int64_t nchunks) {
    const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
    const int x = blockIdx.x % nx;
    const int64_t per = gridDim.x / nx;
    const int64_t lo = nchunks * x / nx, hi = nchunks * (x + 1) / nx;
    return {lo + blockIdx.x / nx, hi, per};
}

template <uint32_t STEPS>
__global__ __launch_bounds__(kMT) void k_mpm(MpmProg mp) {
    constexpr bool G2P = (STEPS & PS_G2P) != 0, ADV = (STEPS & PS_ADVECT) != 0, P2G = (STEPS & PS_P2G) != 0;
    __shared__ float s_tile[3 * kTileMax];         // gather tile [channel][node]
    __shared__ float4 s_stage[kMaxKeys * 27];      // scatter sums [base node][offset]: m, mv
    // scatter records, sorted by base node, one array per field (a thread
    // reading field q of record r hits bank r mod 32)
    __shared__ float s_rec[kRec * kMT];
    __shared__ int32_t s_count[kTileMax];           // particles per base node
    __shared__ int32_t s_first[kTileMax];           // first record of each base node
    __shared__ int32_t s_slot[kTileBlocks];
    __shared__ int32_t s_flag[kTileBlocks];
    __shared__ int s_red[24];
    const int tid = threadIdx.x;
    const int64_t np = mp.np;
    const int64_t nchunks = (np + kMT - 1) / kMT;
    const Chunks ch = chunks_of(nchunks);
    for (int64_t chunk = ch.first; chunk < ch.end; chunk += ch.step) {
        const int64_t p = chunk * kMT + tid;
        const bool valid = p < np;
        float x[3] = {0.f, 0.f, 0.f}, v[3] = {0.f, 0.f, 0.f}, C[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) C[q] = 0.f;
        if (valid)
#pragma unroll
            for (int c = 0; c < 3; ++c) x[c] = mp.x[c * np + p];

        if constexpr (G2P) {
            const GridDev &g = mp.gsrc;
            const int n = g.R * kBS;
            const float inv_dx = mp.inv_dx_src, dx = 1.0f / inv_dx;
            float w[3][3], fx[3];
            int base[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) base[c] = spline(x[c] * inv_dx, w[c], fx[c]);
            const Tile T = tile_of(base, valid, s_red);
            if (T.fits) {
                if (tid < T.blocks) {
                    const int64_t cell = block_cell(g, T, tid);
                    s_slot[tid] = cell >= 0 ? lookup(g, cell) : -1;
                }
                __syncthreads();
                for (int t = tid; t < T.nodes; t += kMT) {
                    const int d = t % T.ext[2], b = (t / T.ext[2]) % T.ext[1], a = t / (T.ext[1] * T.ext[2]);
                    const int i = T.lo[0] + a, j = T.lo[1] + b, k = T.lo[2] + d;
                    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
                    if (in_domain(i, j, k, n)) {
                        const int32_t s = s_slot[tile_block(T, i, j, k)];
                        if (s >= 0) {
                            const int64_t o = (int64_t)s * kBV + voxel_offset(i, j, k);
                            v0 = chan(g, mp.ch_vsrc)[o];
                            v1 = chan(g, mp.ch_vsrc + 1)[o];
                            v2 = chan(g, mp.ch_vsrc + 2)[o];
                        }
                    }
                    s_tile[t] = v0;
                    s_tile[kTileMax + t] = v1;
                    s_tile[2 * kTileMax + t] = v2;
                }
                __syncthreads();
            }
            if (valid) {
                const float kc = 4.0f * inv_dx * inv_dx;
                float B[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) B[q] = 0.f;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const int i = base[0] + a, j = base[1] + b, k = base[2] + d;
                            float vn[3];
                            if (T.fits) {
                                const int t = ((i - T.lo[0]) * T.ext[1] + (j - T.lo[1])) * T.ext[2] + (k - T.lo[2]);
                                vn[0] = s_tile[t];
                                vn[1] = s_tile[kTileMax + t];
                                vn[2] = s_tile[2 * kTileMax + t];
                            } else {
                                vn[0] = vn[1] = vn[2] = 0.f;
                                if (in_domain(i, j, k, n)) {
                                    const int32_t s = lookup(g, ((int64_t)(i >> 3) * g.R + (j >> 3)) * g.R + (k >> 3));
                                    if (s >= 0) {
                                        const int64_t o = (int64_t)s * kBV + voxel_offset(i, j, k);
                                        vn[0] = chan(g, mp.ch_vsrc)[o];
                                        vn[1] = chan(g, mp.ch_vsrc + 1)[o];
                                        vn[2] = chan(g, mp.ch_vsrc + 2)[o];
                                    }
                                }
                            }
                            const float wt = (w[0][a] * w[1][b]) * w[2][d];
                            const float off[3] = {((float)a - fx[0]) * dx, ((float)b - fx[1]) * dx,
                                                  ((float)d - fx[2]) * dx};
#pragma unroll
                            for (int r = 0; r < 3; ++r) {
                                const float wv = wt * vn[r];
                                v[r] = v[r] + wv;
#pragma unroll
                                for (int c = 0; c < 3; ++c) B[3 * r + c] = B[3 * r + c] + wv * off[c];
                            }
                        }
#pragma unroll
                for (int q = 0; q < 9; ++q) C[q] = kc * B[q];
                if (mp.keep & 1u)
#pragma unroll
                    for (int c = 0; c < 3; ++c) mp.v[c * np + p] = v[c];
                if (mp.keep & 2u)
#pragma unroll
                    for (int q = 0; q < 9; ++q) mp.C[q * np + p] = C[q];
            }
            if (P2G) __syncthreads();   // the scatter reuses the tile
        } else if (valid) {
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = mp.v[c * np + p];
            if constexpr (P2G)
#pragma unroll
                for (int q = 0; q < 9; ++q) C[q] = mp.C[q * np + p];
        }

        if constexpr (ADV) {
            if (valid)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    x[c] = x[c] + mp.adv_dt * v[c];
                    mp.x[c * np + p] = x[c];
                }
        }

        if constexpr (P2G) {
            const GridDev &g = mp.gdst;
            const int n = g.R * kBS;
            const float inv_dx = mp.inv_dx_dst, dx = 1.0f / inv_dx;
            // F <- (I + dt C) F, stress, affine momentum matrix A
            float A[9];
            if (valid) {
                float Fo[9], Fn[9], R[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) Fo[q] = mp.F[q * np + p];
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float s = 0.f;
#pragma unroll
                        for (int k = 0; k < 3; ++k) s = s + ((r == k ? 1.0f : 0.0f) + mp.dt * C[3 * r + k]) * Fo[3 * k + c];
                        Fn[3 * r + c] = s;
                    }
#pragma unroll
                for (int q = 0; q < 9; ++q) mp.F[q * np + p] = Fn[q];
                polar_rotation(Fn, R);
                const float J = det3(Fn);
                const float kstress = mp.dt * mp.vol * 4.0f * inv_dx * inv_dx;
                const float vterm = mp.lam * (J - 1.0f) * J;
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float s = 0.f;
#pragma unroll
                        for (int k = 0; k < 3; ++k) s = s + (Fn[3 * r + k] - R[3 * r + k]) * Fn[3 * c + k];
                        const float tau = 2.0f * mp.mu * s + (r == c ? vterm : 0.0f);
                        A[3 * r + c] = -(kstress * tau) + mp.mass * C[3 * r + c];
                    }
            }
            float w[3][3], fx[3];
            int base[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) base[c] = spline(x[c] * inv_dx, w[c], fx[c]);
            const Tile T = tile_of(base, valid, s_red);
            const bool act = mp.act_mode != AT_ACT_NONE;
            const float mvp[3] = {mp.mass * v[0], mp.mass * v[1], mp.mass * v[2]};
            if (T.fits) {
                // base nodes of the chunk: the box [lo, lo + ext - 2) per axis
                const int e0 = T.ext[0] - 2, e1 = T.ext[1] - 2, e2 = T.ext[2] - 2;
                const int nkeys = e0 * e1 * e2;
                for (int t = tid; t < nkeys; t += kMT) s_count[t] = 0;
                if (tid < T.blocks) s_flag[tid] = 0;
                __syncthreads();
                int key = 0, rank = 0;
                if (valid) {
                    key = ((base[0] - T.lo[0]) * e1 + (base[1] - T.lo[1])) * e2 + (base[2] - T.lo[2]);
                    rank = atomicAdd(&s_count[key], 1);
                    // blocks holding the in-domain nodes of the neighbourhood
                    int nlo[3], nhi[3];
                    bool any = true;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        nlo[c] = max(base[c], 0);
                        nhi[c] = min(base[c] + 2, n - 1);
                        any = any && nlo[c] <= nhi[c];
                    }
                    if (any)
                        for (int q = 0; q < 8; ++q) {
                            const int i = (q & 4) ? nhi[0] : nlo[0], j = (q & 2) ? nhi[1] : nlo[1],
                                      k = (q & 1) ? nhi[2] : nlo[2];
                            s_flag[tile_block(T, i, j, k)] = 1;
                        }
                }
                __syncthreads();
                if (tid < T.blocks) {
                    int32_t sl = -1;
                    if (s_flag[tid]) {
                        const int64_t cell = block_cell(g, T, tid);
                        if (cell >= 0) sl = act ? activate(g, cell) : lookup(g, cell);
                    }
                    s_slot[tid] = sl;
                }
                // exclusive scan of the counts (nkeys <= kMaxKeys <= 2 * kMT)
                {
                    const int k0 = 2 * tid;
                    const int c0 = k0 < nkeys ? s_count[k0] : 0, c1 = k0 + 1 < nkeys ? s_count[k0 + 1] : 0;
                    int incl = c0 + c1;
                    const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const int y = __shfl_up(incl, o, 64);
                        if (lane >= o) incl += y;
                    }
                    if (lane == 63) s_red[wid] = incl;
                    __syncthreads();
                    int before = incl - (c0 + c1);
                    for (int w2 = 0; w2 < wid; ++w2) before += s_red[w2];
                    if (k0 < nkeys) s_first[k0] = before;
                    if (k0 + 1 < nkeys) s_first[k0 + 1] = before + c0;
                }
                __syncthreads();
                if (valid) {
                    // fields: fx (3), mass v (3), A (9, row-major)
                    float *r = &s_rec[s_first[key] + rank];
                    r[0] = fx[0];
                    r[kMT] = fx[1];
                    r[2 * kMT] = fx[2];
#pragma unroll
                    for (int c = 0; c < 3; ++c) r[(3 + c) * kMT] = mvp[c];
#pragma unroll
                    for (int q = 0; q < 9; ++q) r[(6 + q) * kMT] = A[q];
                }
                __syncthreads();
                // work items (base node, offset): the four channels' sums of
                // the base's particles at the node base + (a, b, d)
                for (int it = tid; it < 27 * nkeys; it += kMT) {
                    const int kk = it / 27, o = it - 27 * kk;
                    const int a = o / 9, b = (o / 3) % 3, d = o % 3;
                    const int first = s_first[kk], last = first + s_count[kk];
                    float sm = 0.f, s0 = 0.f, s1 = 0.f, s2 = 0.f;
                    for (int r = first; r < last; ++r) {
                        const float *R = s_rec + r;
                        const float f0 = R[0], f1 = R[kMT], f2 = R[2 * kMT];
                        const float t0a = a == 0 ? 1.5f - f0 : a == 1 ? f0 - 1.0f : f0 - 0.5f;
                        const float t0b = b == 0 ? 1.5f - f1 : b == 1 ? f1 - 1.0f : f1 - 0.5f;
                        const float t0d = d == 0 ? 1.5f - f2 : d == 1 ? f2 - 1.0f : f2 - 0.5f;
                        const float wa = a == 1 ? 0.75f - t0a * t0a : 0.5f * (t0a * t0a);
                        const float wb = b == 1 ? 0.75f - t0b * t0b : 0.5f * (t0b * t0b);
                        const float wd = d == 1 ? 0.75f - t0d * t0d : 0.5f * (t0d * t0d);
                        const float wt = (wa * wb) * wd;
                        const float dp0 = ((float)a - f0) * dx, dp1 = ((float)b - f1) * dx, dp2 = ((float)d - f2) * dx;
                        sm += wt * mp.mass;
                        s0 += wt * (R[3 * kMT] + (R[6 * kMT] * dp0 + R[7 * kMT] * dp1 + R[8 * kMT] * dp2));
                        s1 += wt * (R[4 * kMT] + (R[9 * kMT] * dp0 + R[10 * kMT] * dp1 + R[11 * kMT] * dp2));
                        s2 += wt * (R[5 * kMT] + (R[12 * kMT] * dp0 + R[13 * kMT] * dp1 + R[14 * kMT] * dp2));
                    }
                    s_stage[it] = make_float4(sm, s0, s1, s2);
                }
                __syncthreads();
                // one thread per tile node: the staged sums landing on it
                for (int t = tid; t < T.nodes; t += kMT) {
                    const int td = t % T.ext[2], tb = (t / T.ext[2]) % T.ext[1], ta = t / (T.ext[1] * T.ext[2]);
                    const int i = T.lo[0] + ta, j = T.lo[1] + tb, k = T.lo[2] + td;
                    if (!in_domain(i, j, k, n)) continue;
                    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
                    bool hit = false;
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b)
#pragma unroll
                            for (int d = 0; d < 3; ++d) {
                                const int k0 = ta - a, k1 = tb - b, k2 = td - d;
                                if (k0 < 0 || k1 < 0 || k2 < 0 || k0 >= e0 || k1 >= e1 || k2 >= e2) continue;
                                const int kk = (k0 * e1 + k1) * e2 + k2;
                                if (s_count[kk] == 0) continue;
                                const float4 q = s_stage[kk * 27 + (a * 3 + b) * 3 + d];
                                sum.x += q.x;
                                sum.y += q.y;
                                sum.z += q.z;
                                sum.w += q.w;
                                hit = true;
                            }
                    if (!hit) continue;
                    const int32_t sl = s_slot[tile_block(T, i, j, k)];
                    if (sl < 0) continue;
                    const int64_t o = (int64_t)sl * kBV + voxel_offset(i, j, k);
                    atomicAdd(chan(g, mp.ch_m) + o, sum.x);
                    atomicAdd(chan(g, mp.ch_mv) + o, sum.y);
                    atomicAdd(chan(g, mp.ch_mv + 1) + o, sum.z);
                    atomicAdd(chan(g, mp.ch_mv + 2) + o, sum.w);
                }
                __syncthreads();   // the next chunk reuses the LDS arrays
            } else if (valid) {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        for (int d = 0; d < 3; ++d) {
                            const int i = base[0] + a, j = base[1] + b, k = base[2] + d;
                            if (!in_domain(i, j, k, n)) continue;
                            const int64_t cell = ((int64_t)(i >> 3) * g.R + (j >> 3)) * g.R + (k >> 3);
                            const int32_t s = act ? activate(g, cell) : lookup(g, cell);
                            if (s < 0) continue;
                            const float wt = (w[0][a] * w[1][b]) * w[2][d];
                            const float dpos[3] = {((float)a - fx[0]) * dx, ((float)b - fx[1]) * dx,
                                                   ((float)d - fx[2]) * dx};
                            const int64_t o = (int64_t)s * kBV + voxel_offset(i, j, k);
                            atomicAdd(chan(g, mp.ch_m) + o, wt * mp.mass);
                            for (int c = 0; c < 3; ++c) {
                                const float ad = A[3 * c] * dpos[0] + A[3 * c + 1] * dpos[1] + A[3 * c + 2] * dpos[2];
                                atomicAdd(chan(g, mp.ch_mv + c) + o, wt * (mvp[c] + ad));
                            }
                        }
            }
        }
    }
}

}  // namespace

hipError_t launch_mpm(const MpmProg &mp, hipStream_t s) {
    const int64_t nchunks = (mp.np + kMT - 1) / kMT;
    int64_t wgs = 256 * 8;
    if (nchunks < wgs) wgs = nchunks >= 8 ? (nchunks / 8) * 8 : nchunks;
    if (wgs < 1) wgs = 1;
    const dim3 grid((unsigned)wgs), block(kMT);
    switch (mp.steps) {
    case PS_G2P: hipLaunchKernelGGL(k_mpm<PS_G2P>, grid, block, 0, s, mp); break;
    case PS_P2G: hipLaunchKernelGGL(k_mpm<PS_P2G>, grid, block, 0, s, mp); break;
    case PS_G2P | PS_ADVECT: hipLaunchKernelGGL((k_mpm<PS_G2P | PS_ADVECT>), grid, block, 0, s, mp); break;
    case PS_ADVECT | PS_P2G: hipLaunchKernelGGL((k_mpm<PS_ADVECT | PS_P2G>), grid, block, 0, s, mp); break;
    case PS_G2P | PS_P2G: hipLaunchKernelGGL((k_mpm<PS_G2P | PS_P2G>), grid, block, 0, s, mp); break;
    case PS_G2P | PS_ADVECT | PS_P2G:
        hipLaunchKernelGGL((k_mpm<PS_G2P | PS_ADVECT | PS_P2G>), grid, block, 0, s, mp);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ats
