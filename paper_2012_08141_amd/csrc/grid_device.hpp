// Device-side access to a grid's root and leaves, shared by the kernel
// files.  Included inside an unnamed namespace of each, so every file has
// its own internal copies.  Expects internal.hpp (GridDev, header words).
#pragma once

constexpr int kSpinLimit = 1 << 22;      // bounded wait on a pointer-root allocation

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
    // A plain load may return a stale value; staleness only ever shows an
    // active block as inactive (activity never reverts inside a kernel),
    // which sends the thread down the atomic path below -- still correct.
    if (KIND == AT_ROOT_BITMASK) {
        if (!(g.bits[c >> 5] & m)) atomicOr(&g.bits[c >> 5], m);
        return (int32_t)c;
    }
    int32_t s = g.ptr[c];
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

__device__ __forceinline__ void cell_coords(const GridDev &g, int32_t cell, int &bi, int &bj, int &bk) {
    bi = cell / g.R2;
    const int r = cell - bi * g.R2;
    bj = r / g.R;
    bk = r - bj * g.R;
}
