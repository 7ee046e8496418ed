// Runtime-compiled variants of fused element-wise struct-fors.
//
// The paper's engine compiles every fused task it forms from the fused
// kernels' IR, caches the result ("IR bank", an offline cache on disk) and
// compiles in parallel with the program (Sections 5 and 7.2).  This library
// runs fused struct-fors in pre-built kernels; for the programs those cover
// with a per-voxel interpreter (k_micro), this file writes a specialised
// HIP kernel for the node's exact op sequence, compiles it with hiprtc on a
// worker thread (or at first use), keeps the code object in memory and on
// disk, and launches it once it is loaded; until then the interpreter runs
// the node.
//
// Covered: programs of COPY, AXPY, INC, FILL and NORMALISE ops with no
// activation check (the element-wise chains fusion forms).  Within one
// lane's voxels every op of such a program reads and writes at the loop
// index only, so the generated kernel loads each channel it reads before
// writing it once per block, keeps every value in registers from op to op,
// and stores each written channel once:
// the memory it leaves is the interpreter's, with the same arithmetic in
// the same order (compiled without contraction), so results are
// bit-identical.

#include <hip/hip_runtime_api.h>
#include <hip/hiprtc.h>

#include <sys/stat.h>

#include <algorithm>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace ats {
namespace {

constexpr int kMaxVariants = 256;   // beyond this, new programs stay on the interpreter

// hex-float literal of a float (exact), or a builtin for the special values
std::string flit(float v) {
    char b[64];
    if (v != v) return "__builtin_nanf(\"\")";
    if (v == __builtin_inff()) return "__builtin_inff()";
    if (v == -__builtin_inff()) return "(-__builtin_inff())";
    std::snprintf(b, sizeof b, "%af", (double)v);
    return b;
}

bool op_supported(const MicroOp &op) {
    return op.op == AT_OP_COPY || op.op == AT_OP_AXPY || op.op == AT_OP_INC || op.op == AT_OP_FILL ||
           op.op == AT_OP_NORMALISE;
}

// Kernel source for one program.  Same loop over list records and lane
// layout as the interpreter (one wavefront per block, lane l owning the
// voxels 8l .. 8l + 7 as two float4 halves, suffixes a and b), but written
// in the order the memory system wants: every channel the program reads
// before writing it is loaded once per block, both halves at once; the next
// block's loads are issued before the current block's stores (blocks are
// disjoint, so this is safe; a compiler cannot know it); the ops run on
// registers; each written channel is stored once.
struct Gen {
    std::vector<int> loads;      // channels read before any op writes them, in order
    std::map<int, bool> have;    // channels with a register value
    std::vector<int> written;    // channels written, in order of first write
    std::string body;            // compute code for one half, '@' for the suffix

    static std::string var(int c) { return "c" + std::to_string(c) + "@"; }
    std::string get(int c) {
        if (!have.count(c)) {
            loads.push_back(c);
            have[c] = true;
        }
        return var(c);
    }
    void set(int c, const std::string &expr) {
        have[c] = true;
        if (std::find(written.begin(), written.end(), c) == written.end()) written.push_back(c);
        body += "        " + var(c) + " = " + expr + ";\n";
    }
};

std::string subst(const std::string &code, char h) {
    std::string r = code;
    for (char &ch : r)
        if (ch == '@') ch = h;
    return r;
}

std::string generate(const MicroProg &prog) {
    Gen G;
    for (int o = 0; o < prog.nops; ++o) {
        const MicroOp &op = prog.ops[o];
        const std::string p = flit(op.p);
        switch (op.op) {
        case AT_OP_COPY: {
            const std::string x = G.get(op.ch[1]);
            G.set(op.ch[0], x);
            break;
        }
        case AT_OP_AXPY: {
            const std::string y = G.get(op.ch[0]), x = G.get(op.ch[1]);
            G.body += "        t.x = " + y + ".x + " + p + " * " + x + ".x; t.y = " + y + ".y + " + p + " * " + x +
                      ".y; t.z = " + y + ".z + " + p + " * " + x + ".z; t.w = " + y + ".w + " + p + " * " + x + ".w;\n";
            G.set(op.ch[0], "t");
            break;
        }
        case AT_OP_INC: {
            const std::string x = G.get(op.ch[0]);
            G.body += "        t.x = " + x + ".x + " + p + "; t.y = " + x + ".y + " + p + "; t.z = " + x + ".z + " + p +
                      "; t.w = " + x + ".w + " + p + ";\n";
            G.set(op.ch[0], "t");
            break;
        }
        case AT_OP_FILL:
            for (int q = 0; q < 7; ++q)
                if (op.ch[q] >= 0 && ((op.keep >> q) & 1u))
                    G.set(op.ch[q], "make_float4(" + p + ", " + p + ", " + p + ", " + p + ")");
            break;
        case AT_OP_NORMALISE: {
            const std::string m = G.get(op.ch[0]);
            for (int cc = 0; cc < 3; ++cc) {
                if (!((op.keep >> cc) & 1u)) continue;
                const std::string mv = G.get(op.ch[1] + cc);
                G.body += "        t.x = " + m + ".x > 0.f ? " + mv + ".x / " + m + ".x : 0.f; t.y = " + m + ".y > 0.f ? " +
                          mv + ".y / " + m + ".y : 0.f; t.z = " + m + ".z > 0.f ? " + mv + ".z / " + m + ".z : 0.f; t.w = " +
                          m + ".w > 0.f ? " + mv + ".w / " + m + ".w : 0.f;\n";
                G.set(op.ch[2] + cc, "t");
            }
            break;
        }
        default:
            break;
        }
    }
    auto ld = [](int c, const char *o, const char *h) {
        return std::string("*reinterpret_cast<const float4 *>(ch + ") + std::to_string(c) + "LL * stride + " + o +
               (h[0] == 'b' ? " + 4" : "") + ")";
    };
    std::string s;
    s += "#include <hip/hip_runtime.h>\n";
    s += "extern \"C\" __global__ __launch_bounds__(64) void atsv(const int *__restrict__ hdr, const int *__restrict__ "
         "list, float *__restrict__ ch, long long stride) {\n";
    s += "    const int lane = threadIdx.x;\n";
    s += "    const int count = hdr[" + std::to_string(HDR_COUNT) + "];\n";
    s += "    const int nx = (gridDim.x % 8 == 0) ? 8 : 1;\n";
    s += "    const int xs = blockIdx.x % nx;\n";
    s += "    const int lo = (int)(((long long)count * xs) / nx) + (int)(blockIdx.x / nx);\n";
    s += "    const int hi = (int)(((long long)count * (xs + 1)) / nx);\n";
    s += "    const int step = gridDim.x / nx;\n";
    s += "    if (lo >= hi) return;\n";
    s += "    long long off = (long long)list[(long long)lo * " + std::to_string(kRec) + " + 1] * " +
         std::to_string(kBV) + " + lane * 8;\n";
    for (int c : G.loads)
        for (const char *h : {"a", "b"}) s += "    float4 p" + std::to_string(c) + h + " = " + ld(c, "off", h) + ";\n";
    s += "    for (int e = lo; e < hi; e += step) {\n";
    s += "        const int en = e + step < hi ? e + step : e;\n";
    s += "        const long long offn = (long long)list[(long long)en * " + std::to_string(kRec) + " + 1] * " +
         std::to_string(kBV) + " + lane * 8;\n";
    for (int c : G.loads)
        for (const char *h : {"a", "b"}) s += "        const float4 n" + std::to_string(c) + h + " = " + ld(c, "offn", h) + ";\n";
    s += "        float4 t;\n";
    for (const auto &kv : G.have) {
        const bool loaded = std::find(G.loads.begin(), G.loads.end(), kv.first) != G.loads.end();
        for (const char *h : {"a", "b"})
            s += "        float4 c" + std::to_string(kv.first) + h +
                 (loaded ? " = p" + std::to_string(kv.first) + h : std::string()) + ";\n";
    }
    s += subst(G.body, 'a');
    s += subst(G.body, 'b');
    for (int c : G.written)
        for (const char *h : {"a", "b"})
            s += std::string("        *reinterpret_cast<float4 *>(ch + ") + std::to_string(c) + "LL * stride + off" +
                 (h[0] == 'b' ? " + 4" : "") + ") = c" + std::to_string(c) + h + ";\n";
    for (int c : G.loads)
        for (const char *h : {"a", "b"}) s += "        p" + std::to_string(c) + h + " = n" + std::to_string(c) + h + ";\n";
    s += "        off = offn;\n";
    s += "    }\n}\n";
    return s;
}

// ------------------------------------------------ advection tile programs
// A tile program (sampling ops with element-wise ops beside them, see
// k_tile_micro) compiled for its exact op sequence: the same staging of the
// block and its 2-voxel halo in LDS, the same back-traces, clamps, corner
// weights, corner order and sums, but with the ops written out instead of
// interpreted (no per-op descriptor loads, constants in the code, only the
// live values in registers), so results are bit-identical to k_tile_micro.
const char *kTilePrelude = R"(constexpr int kBS = 8, kBV = 512, kRec = 8, kTE = 12, kT3 = kTE * kTE * kTE, kTC = 3;
struct G {
    const unsigned *bits;
    const int *ptr;
    float *chan;
    long long stride;
    int R, R2;
};
__device__ __forceinline__ float *chan(const G &g, int c) { return g.chan + (long long)c * g.stride; }
__device__ __forceinline__ int slot_of(const G &g, long long c) {
#if KIND == 0
    return ((g.bits[c >> 5] >> (c & 31)) & 1u) ? (int)c : -1;
#else
    const int s = g.ptr[c];
    return s >= 0 ? s : -1;
#endif
}
__device__ __forceinline__ float clamp_coord(float p, int n) {
    return p < -2.f ? -2.f : (p > (float)(n + 1) ? (float)(n + 1) : p);
}
__device__ __forceinline__ float sample_voxel(const G &g, const float *base, long long own_cell, int own_slot, int x,
                                              int y, int z, int n) {
    if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return 0.f;
    const long long c = ((long long)(x >> 3) * g.R + (y >> 3)) * g.R + (z >> 3);
    const int s = c == own_cell ? own_slot : slot_of(g, c);
    return s >= 0 ? base[(long long)s * kBV + (x & 7) * 64 + (y & 7) * 8 + (z & 7)] : 0.f;
}
__device__ __forceinline__ float sample_far(const G &g, const float *base, long long cell, int slot, const float p[3],
                                            int n) {
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
        acc = acc + wt * sample_voxel(g, base, cell, slot, b0[0] + a, b0[1] + b, b0[2] + c, n);
    }
    return acc;
}
__device__ __forceinline__ void corners_far(const G &g, const float *Q, long long cell, int slot, const float p[3],
                                            int n, float &lo, float &hi) {
    int b0[3];
    for (int d = 0; d < 3; ++d) b0[d] = (int)floorf(clamp_coord(p[d], n));
#pragma nounroll
    for (int q = 0; q < 8; ++q) {
        const float x = sample_voxel(g, Q, cell, slot, b0[0] + (q >> 2), b0[1] + ((q >> 1) & 1), b0[2] + (q & 1), n);
        if (q == 0) {
            lo = x;
            hi = x;
        } else {
            lo = x < lo ? x : lo;
            hi = x > hi ? x : hi;
        }
    }
}
__device__ __forceinline__ float sample_staged(const G &g, const float *T, const int o[3], const float *base,
                                               long long cell, int slot, const float p[3], int n) {
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
    if (!in) return sample_far(g, base, cell, slot, p, n);
    float acc = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                const float wt = (w[0][a] * w[1][b]) * w[2][c];
                acc = acc + wt * T[((lb[0] + a) * kTE + (lb[1] + b)) * kTE + (lb[2] + c)];
            }
    return acc;
}
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
__device__ __forceinline__ float tile_sum(const float *T, const float wt[8]) {
    float acc = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) acc = acc + wt[(a * 2 + b) * 2 + c] * T[(a * kTE + b) * kTE + c];
    return acc;
}
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
    const int bk = d2 ? 1 : 3, bj = d1 ? 1 : 3;
    const int sk = l & ((1 << bk) - 1), sj = (l >> bk) & ((1 << bj) - 1), si = l >> (bk + bj);
    const int i = d0 < 0 ? 6 + si : si, j = d1 < 0 ? 6 + sj : sj, k = d2 < 0 ? 6 + sk : sk;
    src = i * 64 + j * 8 + k;
    const int ti = d0 < 0 ? si : (d0 ? 10 + si : 2 + si), tj = d1 < 0 ? sj : (d1 ? 10 + sj : 2 + sj),
              tk = d2 < 0 ? sk : (d2 ? 10 + sk : 2 + sk);
    tpos = (ti * kTE + tj) * kTE + tk;
    return (d0 + 1) * 9 + (d1 + 1) * 3 + (d2 + 1);
}
extern "C" __global__ __launch_bounds__(kTT) void atst(const unsigned *bits, const int *ptr, const int *list,
                                                        const int *hdr, float *chanb, long long stride, int R) {
    extern __shared__ float s_t[];
    __shared__ int s_nb[27];
    const G g{bits, ptr, chanb, stride, R, R * R};
    const int tid = threadIdx.x;
    const int n = R * kBS;
    float *vs = s_t + NT * kT3;
    const int count = hdr[HDR_COUNT];
    const int nx = (gridDim.x % 8 == 0) ? 8 : 1;
    const int xs = blockIdx.x % nx;
    const int lo = (int)(((long long)count * xs) / nx) + (int)(blockIdx.x / nx);
    const int hi = (int)(((long long)count * (xs + 1)) / nx);
    const int step = gridDim.x / nx;
    static_assert(kTT == kBV, "one voxel per thread");
    // slot of neighbour t (0 .. 26) of the block listed at e, -1 outside the
    // domain or inactive
    auto nb_slot = [&](int e, int t) {
        const int2 r = *reinterpret_cast<const int2 *>(list + (long long)e * kRec);
        const int b0 = r.x / g.R2, b1 = (r.x - b0 * g.R2) / R, b2 = r.x - b0 * g.R2 - b1 * R;
        const int ni = b0 + t / 9 - 1, nj = b1 + (t / 3) % 3 - 1, nk = b2 + t % 3 - 1;
        int sl = -1;
        if (ni >= 0 && nj >= 0 && nk >= 0 && ni < R && nj < R && nk < R)
            sl = t == 13 ? r.y : slot_of(g, ((long long)ni * R + nj) * R + nk);
        return sl;
    };
    if (lo < hi && tid < 27) s_nb[tid] = nb_slot(lo, tid);
    __syncthreads();
    for (int e = lo; e < hi; e += step) {
        const int4 rec0 = *reinterpret_cast<const int4 *>(list + (long long)e * kRec);
        const int cell = rec0.x, slot = rec0.y;
        const int bi = cell / g.R2, rr = cell - bi * g.R2, bj = rr / R, bk = rr - bj * R;
        // the block's own velocity, loaded with the first staging chunk
#if VOWN
        float vo[3];
        for (int d = 0; d < 3; ++d) vo[d] = chan(g, V0 + d)[(long long)slot * kBV + tid];
#endif
        constexpr int NIT = (kT3 + kTT - 1) / kTT;
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
                const int sl = s_nb[tile_src(t, src, tpos[u])];
                ok[u] = sl >= 0;
                const long long o = (long long)(sl >= 0 ? sl : slot) * kBV + src;
#pragma unroll
                for (int q = 0; q < NC; ++q) val[u][q] = chan(g, stage_ch(q))[o];
            }
#pragma unroll
            for (int u = 0; u < kTC; ++u) {
                const int it = c0 + u;
                if (it >= NIT) break;
                if (tid + it * kTT < kT3) {
#pragma unroll
                    for (int q = 0; q < NC; ++q) s_t[q * kT3 + tpos[u]] = ok[u] ? val[u][q] : 0.f;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#if VOWN
        for (int d = 0; d < 3; ++d) vs[d * kBV + tid] = vo[d];
#endif
        __syncthreads();
        // the next block's neighbour slots, looked up while this block computes
        // (the staging above was their last reader)
        const int en = e + step;
        int nbn = -1;
        if (tid < 27 && en < hi) nbn = nb_slot(en, tid);
        const int org[3] = {bi * kBS - 2, bj * kBS - 2, bk * kBS - 2};
#pragma nounroll
        for (int vx = tid; vx < kBV; vx += kTT) {
            // lanes permuted within the wave's 8x8 plane (rows 0, 2, 4, 6 in the first half, 1, 3, 5, 7
            // in the second), so that its corner reads at a common offset fall in distinct LDS banks
            const int li = vx >> 6, lj = ((vx >> 3) & 3) * 2 + ((vx >> 5) & 1), lk = vx & 7;
            const int vm = li * 64 + lj * 8 + lk;
            const int I[3] = {bi * kBS + li, bj * kBS + lj, bk * kBS + lk};
            const long long off = (long long)slot * kBV + vm;
            (void)I;
            (void)org;
)";

// Source of the tile program's variant for root kind `kind`.
std::string generate_tile(const TileProg &tp, int kind) {
    const MicroProg &prog = tp.prog;
    std::string s = "#include <hip/hip_runtime.h>\n#define KIND " + std::to_string(kind) + "\n";
    s += "#define HDR_COUNT " + std::to_string(HDR_COUNT) + "\n";
    s += "constexpr int kTT = " + std::to_string(kTT) + ";\n";
    s += "constexpr int NT = " + std::to_string(tp.nt) + ";\n";
    const int nc = tp.nt + (tp.vstage ? 3 : 0);
    s += "constexpr int NC = " + std::to_string(nc) + ";\n";
    s += "#define V0 " + std::to_string(tp.v0) + "\n";
    s += "#define VOWN " + std::string(!tp.vstage && tp.v0 >= 0 ? "1" : "0") + "\n";
    // the staged channels: the sampled ones, then the velocity tiles
    s += "__device__ __forceinline__ constexpr int stage_ch(int q) { return ";
    for (int q = 0; q < nc; ++q) {
        const int c = q < tp.nt ? tp.tch[q] : tp.v0 + (q - tp.nt);
        s += "q == " + std::to_string(q) + " ? " + std::to_string(c) + " : ";
    }
    s += "-1; }\n";
    s += kTilePrelude;
    auto staged = [&](int ch) {
        for (int q = 0; q < tp.nt; ++q)
            if (tp.tch[q] == ch) return q;
        return -1;
    };
    auto C = [](int c) { return "chan(g, " + std::to_string(c) + ")"; };
    std::string b;
    // the back-trace of the last (velocity, dt, rk3), as the interpreter keeps it
    int pv = -1, ntr = 0;
    float pdt = 0.f, prk = -1.f;
    std::string T;   // current trace's variable prefix
    for (int o = 0; o < prog.nops; ++o) {
        const MicroOp &op = prog.ops[o];
        const std::string P = flit(op.p);
        if (op.op == AT_OP_ADVECT || op.op == AT_OP_MACCORMACK) {
            if (!(op.ch[1] == pv && op.p == pdt && op.p1 == prk)) {
                T = "t" + std::to_string(ntr++) + "_";
                b += "            float " + T + "v1[3], " + T + "pt[3], " + T + "wt[8];\n";
                b += "            for (int d = 0; d < 3; ++d) " + T + "v1[d] = ";
                if (op.ch[1] == tp.v0 && tp.vstage) b += "vs[d * kT3 + ((li + 2) * kTE + (lj + 2)) * kTE + (lk + 2)];\n";
                else if (op.ch[1] == tp.v0) b += "vs[d * kBV + vm];\n";
                else b += "chan(g, " + std::to_string(op.ch[1]) + " + d)[off];\n";
                if (!tp.vstage || op.p1 == 0.f) {
                    b += "            for (int d = 0; d < 3; ++d) " + T + "pt[d] = (float)I[d] - " + P + " * " + T + "v1[d];\n";
                } else {
                    const std::string vt = op.ch[1] == tp.v0 ? "vs" : "";
                    b += "            {\n";
                    b += "                const float h1 = 0.5f * " + P + ", h2 = 0.75f * " + P + ";\n";
                    b += "                float p1[3], v2[3], p2[3], v3[3];\n";
                    b += "                for (int d = 0; d < 3; ++d) p1[d] = (float)I[d] - h1 * " + T + "v1[d];\n";
                    b += "                for (int d = 0; d < 3; ++d) v2[d] = sample_staged(g, " +
                         (vt.empty() ? std::string("nullptr") : "vs + d * kT3") + ", org, chan(g, " +
                         std::to_string(op.ch[1]) + " + d), cell, slot, p1, n);\n";
                    b += "                for (int d = 0; d < 3; ++d) p2[d] = (float)I[d] - h2 * v2[d];\n";
                    b += "                for (int d = 0; d < 3; ++d) v3[d] = sample_staged(g, " +
                         (vt.empty() ? std::string("nullptr") : "vs + d * kT3") + ", org, chan(g, " +
                         std::to_string(op.ch[1]) + " + d), cell, slot, p2, n);\n";
                    b += "                const float c1 = (float)(2.0 / 9.0), c2 = (float)(1.0 / 3.0), c3 = (float)(4.0 / 9.0);\n";
                    b += "                for (int d = 0; d < 3; ++d) {\n";
                    b += "                    float sv = c1 * " + T + "v1[d];\n";
                    b += "                    sv = sv + c2 * v2[d];\n";
                    b += "                    sv = sv + c3 * v3[d];\n";
                    b += "                    " + T + "pt[d] = (float)I[d] - " + P + " * sv;\n";
                    b += "                }\n";
                    b += "            }\n";
                }
                b += "            const int " + T + "lb = trace_tile(" + T + "pt, org, n, " + T + "wt);\n";
                pv = op.ch[1];
                pdt = op.p;
                prk = op.p1;
            }
            const int q = staged(op.ch[0]);
            const std::string tile = q >= 0 ? "s_t + " + std::to_string(q) + " * kT3 + " + T + "lb" : "";
            if (op.op == AT_OP_ADVECT) {
                b += "            " + C(op.ch[2]) + "[off] = ";
                if (q >= 0)
                    b += T + "lb >= 0 ? tile_sum(" + tile + ", " + T + "wt) : sample_far(g, " + C(op.ch[0]) +
                         ", cell, slot, " + T + "pt, n);\n";
                else
                    b += "sample_far(g, " + C(op.ch[0]) + ", cell, slot, " + T + "pt, n);\n";
            } else {
                b += "            {\n";
                b += "                float lo = 0.f, hi = 0.f;\n";
                if (q >= 0) {
                    b += "                if (" + T + "lb >= 0) {\n";
                    b += "                    const float *Tq = " + tile + ";\n";
                    b += "                    for (int a = 0; a < 2; ++a)\n";
                    b += "                        for (int bb = 0; bb < 2; ++bb)\n";
                    b += "                            for (int c = 0; c < 2; ++c) {\n";
                    b += "                                const float x = Tq[(a * kTE + bb) * kTE + c];\n";
                    b += "                                if (a + bb + c == 0) {\n";
                    b += "                                    lo = x;\n";
                    b += "                                    hi = x;\n";
                    b += "                                } else {\n";
                    b += "                                    lo = x < lo ? x : lo;\n";
                    b += "                                    hi = x > hi ? x : hi;\n";
                    b += "                                }\n";
                    b += "                            }\n";
                    b += "                } else {\n";
                    b += "                    corners_far(g, " + C(op.ch[0]) + ", cell, slot, " + T + "pt, n, lo, hi);\n";
                    b += "                }\n";
                } else {
                    b += "                corners_far(g, " + C(op.ch[0]) + ", cell, slot, " + T + "pt, n, lo, hi);\n";
                }
                b += "                const float dq = " + C(op.ch[0]) + "[off] - " + C(op.ch[3]) + "[off];\n";
                b += "                const float h2 = 0.5f * dq;\n";
                b += "                const float val = " + C(op.ch[2]) + "[off] + h2;\n";
                b += "                " + C(op.ch[4]) + "[off] = val < lo ? lo : (val > hi ? hi : val);\n";
                b += "            }\n";
            }
        } else if (op.op == AT_OP_COPY) {
            b += "            " + C(op.ch[0]) + "[off] = " + C(op.ch[1]) + "[off];\n";
        } else if (op.op == AT_OP_AXPY) {
            b += "            " + C(op.ch[0]) + "[off] = " + C(op.ch[0]) + "[off] + " + P + " * " + C(op.ch[1]) + "[off];\n";
        } else if (op.op == AT_OP_INC) {
            b += "            " + C(op.ch[0]) + "[off] = " + C(op.ch[0]) + "[off] + " + P + ";\n";
        } else if (op.op == AT_OP_FILL) {
            for (int qq = 0; qq < 7; ++qq)
                if (op.ch[qq] >= 0 && ((op.keep >> qq) & 1u)) b += "            " + C(op.ch[qq]) + "[off] = " + P + ";\n";
        }
    }
    s += b;
    s += "        }\n        if (tid < 27 && en < hi) s_nb[tid] = nbn;\n        __syncthreads();\n    }\n}\n";
    return s;
}

uint64_t hash_text(const std::string &s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

const char *kOpts[] = {"--offload-arch=gfx950", "-O3", "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
                       "-packed-fp32-ops"};
constexpr int kNOpts = sizeof kOpts / sizeof kOpts[0];

std::string cache_dir() {
    const char *x = std::getenv("XDG_CACHE_HOME");
    std::string base = x && *x ? std::string(x) : (std::getenv("HOME") ? std::string(std::getenv("HOME")) + "/.cache" : "");
    if (base.empty()) return "";
    return base + "/atsparse/variants";
}

bool read_file(const std::string &path, std::vector<char> &out) {
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::fseek(f, 0, SEEK_END);
    const long n = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    out.resize(n > 0 ? (size_t)n : 0);
    const bool ok = n > 0 && std::fread(out.data(), 1, out.size(), f) == out.size();
    std::fclose(f);
    return ok;
}

void write_file(const std::string &dir, const std::string &path, const std::vector<char> &data) {
    std::string d;
    for (size_t i = 0; i <= dir.size(); ++i) {   // mkdir -p
        if (i == dir.size() || dir[i] == '/') {
            if (!d.empty()) ::mkdir(d.c_str(), 0755);
        }
        if (i < dir.size()) d += dir[i];
    }
    const std::string tmp = path + ".tmp" + std::to_string((unsigned long)std::hash<std::thread::id>()(std::this_thread::get_id()));
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    const bool ok = std::fwrite(data.data(), 1, data.size(), f) == data.size();
    std::fclose(f);
    if (ok) std::rename(tmp.c_str(), path.c_str());
    else std::remove(tmp.c_str());
}

// Compiles (or reads from the disk cache) one variant's code object.
bool build_code(uint64_t key, const std::string &src, std::vector<char> &code, bool &from_disk) {
    char name[32];
    std::snprintf(name, sizeof name, "%016llx.co", (unsigned long long)key);
    const std::string dir = cache_dir();
    from_disk = false;
    if (!dir.empty() && read_file(dir + "/" + name, code)) {
        from_disk = true;
        return true;
    }
    hiprtcProgram p;
    if (hiprtcCreateProgram(&p, src.c_str(), "variant.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) return false;
    bool ok = hiprtcCompileProgram(p, kNOpts, kOpts) == HIPRTC_SUCCESS;
    size_t n = 0;
    if (ok) ok = hiprtcGetCodeSize(p, &n) == HIPRTC_SUCCESS && n > 0;
    if (ok) {
        code.resize(n);
        ok = hiprtcGetCode(p, code.data()) == HIPRTC_SUCCESS;
    }
    hiprtcDestroyProgram(&p);
    if (ok && !dir.empty()) write_file(dir, dir + "/" + name, code);
    return ok;
}

// Key of a variant: the program's ops, channels, constants and keep masks
// (what the generated source is a function of), the compile options and
// the generator's revision (bumped whenever the generated code's form
// changes).  Computed from the program's fields, so a launch that finds its
// variant loaded generates no source.
constexpr const char *kGenRevision = "atsv-4";
uint64_t variant_key(const MicroProg &prog) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint32_t v) {
        for (int b = 0; b < 4; ++b) {
            h ^= (v >> (8 * b)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    mix((uint32_t)prog.nops);
    for (int o = 0; o < prog.nops; ++o) {
        const MicroOp &op = prog.ops[o];
        uint32_t pb;
        std::memcpy(&pb, &op.p, 4);
        mix((uint32_t)op.op);
        for (int c = 0; c < 7; ++c) mix((uint32_t)op.ch[c]);
        mix(pb);
        mix(op.keep);
    }
    std::string k;
    for (int i = 0; i < kNOpts; ++i) k += std::string(" ") + kOpts[i];
    return h ^ (hash_text(k + kGenRevision) * 0x9e3779b97f4a7c15ull);
}

// Key of a tile program's variant: every field of its ops (the trace
// parameters included), the root kind and the workgroup size.
constexpr const char *kTileRevision = "atst-3";
uint64_t tile_key(const MicroProg &prog, int kind) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint32_t v) {
        for (int b = 0; b < 4; ++b) {
            h ^= (v >> (8 * b)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    auto mixf = [&](float f) {
        uint32_t u;
        std::memcpy(&u, &f, 4);
        mix(u);
    };
    mix((uint32_t)prog.nops);
    mix((uint32_t)kind);
    mix((uint32_t)kTT);
    for (int o = 0; o < prog.nops; ++o) {
        const MicroOp &op = prog.ops[o];
        mix((uint32_t)op.op);
        for (int c = 0; c < 7; ++c) mix((uint32_t)op.ch[c]);
        mixf(op.p);
        mixf(op.p1);
        mixf(op.p2);
        mix(op.keep);
    }
    std::string k;
    for (int i = 0; i < kNOpts; ++i) k += std::string(" ") + kOpts[i];
    return h ^ (hash_text(k + kTileRevision) * 0x9e3779b97f4a7c15ull);
}

struct Variant {
    enum State { QUEUED, READY, FAILED } state = QUEUED;
    std::string src;
    std::vector<char> code;
    bool from_disk = false;
    int device = -1;
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
};

struct Variants {
    std::mutex mu;
    std::condition_variable cv;
    std::unordered_map<uint64_t, Variant> map;
    std::deque<uint64_t> queue;     // keys waiting for the compile thread
    bool worker = false;
    int mode = 0;                   // 0 off, 1 background compile, 2 compile at first use
    int64_t loaded = 0, compiled = 0, disk_hits = 0;
};

Variants &V() {
    static Variants *v = new Variants();
    return *v;
}

void compile_loop() {
    Variants &v = V();
    for (;;) {
        uint64_t key;
        std::string src;
        {
            std::unique_lock<std::mutex> lk(v.mu);
            v.cv.wait(lk, [&] { return !v.queue.empty(); });
            key = v.queue.front();
            v.queue.pop_front();
            src = v.map[key].src;
        }
        std::vector<char> code;
        bool disk = false;
        const bool ok = build_code(key, src, code, disk);
        std::lock_guard<std::mutex> lk(v.mu);
        Variant &var = v.map[key];
        var.state = ok ? Variant::READY : Variant::FAILED;
        var.code.swap(code);
        var.from_disk = disk;
        if (ok) (disk ? v.disk_hits : v.compiled) += 1;
        v.cv.notify_all();
    }
}

}  // namespace

// Memory accesses per voxel: the interpreter's (each op reads its inputs
// and writes its outputs) and the variant's (each channel read before being
// written loaded once, each written channel stored once).
static void accesses(const MicroProg &prog, int &interp, int &variant) {
    std::map<int, int> state;   // 1 read first, 2 written
    int loads = 0;
    interp = 0;
    auto rd = [&](int c) {
        ++interp;
        if (!state.count(c)) {
            state[c] = 1;
            ++loads;
        }
    };
    auto wr = [&](int c) {
        ++interp;
        state[c] = 2;
    };
    for (int o = 0; o < prog.nops; ++o) {
        const MicroOp &op = prog.ops[o];
        switch (op.op) {
        case AT_OP_COPY: rd(op.ch[1]); wr(op.ch[0]); break;
        case AT_OP_AXPY: rd(op.ch[0]); rd(op.ch[1]); wr(op.ch[0]); break;
        case AT_OP_INC: rd(op.ch[0]); wr(op.ch[0]); break;
        case AT_OP_FILL:
            for (int q = 0; q < 7; ++q)
                if (op.ch[q] >= 0 && ((op.keep >> q) & 1u)) wr(op.ch[q]);
            break;
        case AT_OP_NORMALISE:
            rd(op.ch[0]);
            for (int cc = 0; cc < 3; ++cc)
                if ((op.keep >> cc) & 1u) {
                    rd(op.ch[1] + cc);
                    wr(op.ch[2] + cc);
                }
            break;
        default: break;
        }
    }
    int stores = 0;
    for (const auto &kv : state) stores += kv.second == 2;
    variant = loads + stores;
}

// A variant pays when it saves memory traffic: measured on MI355X, a chain
// whose variant moves as many bytes as the interpreter (three copies, a copy
// and an axpy) runs slower as a variant (the interpreter streams such chains
// at about 5.3 TB/s), while chains of 8 and 16 ops ran 2.9x and 5.7x faster.
bool variant_eligible(const MicroProg &prog) {
    if (prog.check || prog.nops < 2) return false;
    for (int o = 0; o < prog.nops; ++o)
        if (!op_supported(prog.ops[o])) return false;
    int interp, variant;
    accesses(prog, interp, variant);
    return 2 * interp >= 3 * variant;
}

bool variant_launch(const GridDev &g, const MicroProg &prog, hipStream_t s, hipError_t &err) {
    err = hipSuccess;
    Variants &v = V();
    int mode;
    {
        std::lock_guard<std::mutex> lk(v.mu);
        mode = v.mode;
    }
    if (mode == 0) return false;
    TileProg tp;
    const bool elem = variant_eligible(prog);
    const bool tile = !elem && tile_prog(prog, tp);
    if (!elem && !tile) return false;
    const uint64_t key = tile ? tile_key(prog, g.kind) : variant_key(prog);
    hipFunction_t fn = nullptr;
    {
        std::unique_lock<std::mutex> lk(v.mu);
        auto it = v.map.find(key);
        if (it == v.map.end()) {
            if ((int64_t)v.map.size() >= kMaxVariants) return false;
            const std::string src = tile ? generate_tile(tp, g.kind) : generate(prog);
            Variant &nv = v.map[key];
            nv.src = src;
            if (mode == 2) {
                // compile here, at first use
                lk.unlock();
                std::vector<char> code;
                bool disk = false;
                const bool ok = build_code(key, src, code, disk);
                lk.lock();
                Variant &var = v.map[key];
                var.state = ok ? Variant::READY : Variant::FAILED;
                var.code.swap(code);
                var.from_disk = disk;
                if (ok) (disk ? v.disk_hits : v.compiled) += 1;
                v.cv.notify_all();
            } else {
                if (!v.worker) {
                    std::thread(compile_loop).detach();
                    v.worker = true;
                }
                v.queue.push_back(key);
                v.cv.notify_all();
                return false;
            }
            it = v.map.find(key);
        }
        Variant &var = it->second;
        if (var.state == Variant::QUEUED && mode == 2) {
            v.cv.wait(lk, [&] { return v.map[key].state != Variant::QUEUED; });
        }
        if (var.state != Variant::READY) return false;
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        if (!var.fn || var.device != dev) {
            hipModule_t mod = nullptr;
            hipFunction_t f = nullptr;
            if (hipModuleLoadData(&mod, var.code.data()) != hipSuccess ||
                hipModuleGetFunction(&f, mod, tile ? "atst" : "atsv") != hipSuccess) {
                (void)hipGetLastError();
                if (mod) (void)hipModuleUnload(mod);
                var.state = Variant::FAILED;
                return false;
            }
            var.mod = mod;
            var.fn = f;
            var.device = dev;
            v.loaded += 1;
        }
        fn = var.fn;
    }
    const int32_t *hdr = g.hdr;
    const int32_t *list = g.list;
    float *ch = g.chan;
    long long stride = (long long)g.ch_stride;
    if (tile) {
        const uint32_t *bits = g.bits;
        const int32_t *ptr = g.ptr;
        int R = g.R;
        void *args[] = {(void *)&bits, (void *)&ptr, (void *)&list, (void *)&hdr, (void *)&ch, (void *)&stride, (void *)&R};
        const size_t lds = tile_lds_bytes(tp);
        err = hipModuleLaunchKernel(fn, tile_grid_size(g, lds), 1, 1, kTT, 1, 1, (unsigned)lds, s, args, nullptr);
        return true;
    }
    void *args[] = {(void *)&hdr, (void *)&list, (void *)&ch, (void *)&stride};
    err = hipModuleLaunchKernel(fn, (unsigned)wave_grid_size(g, false), 1, 1, 64, 1, 1, 0, s, args, nullptr);
    return true;
}

void set_variant_mode(int mode) {
    std::lock_guard<std::mutex> lk(V().mu);
    V().mode = mode;
}

int variant_mode() {
    std::lock_guard<std::mutex> lk(V().mu);
    return V().mode;
}

int64_t variants_loaded() {
    std::lock_guard<std::mutex> lk(V().mu);
    return V().loaded;
}

bool variant_prepare(const MicroProg &prog, int kind, std::string &src) {
    TileProg tp;
    const bool elem = variant_eligible(prog);
    if (!elem && !tile_prog(prog, tp)) return false;
    src = elem ? generate(prog) : generate_tile(tp, kind);
    const uint64_t key = elem ? variant_key(prog) : tile_key(prog, kind);
    Variants &v = V();
    {
        std::unique_lock<std::mutex> lk(v.mu);
        auto it = v.map.find(key);
        if (it != v.map.end()) {
            v.cv.wait(lk, [&] { return v.map[key].state != Variant::QUEUED; });
            return v.map[key].state == Variant::READY;
        }
        if ((int64_t)v.map.size() >= kMaxVariants) return false;
        v.map[key].src = src;
    }
    std::vector<char> code;
    bool disk = false;
    const bool ok = build_code(key, src, code, disk);
    std::lock_guard<std::mutex> lk(v.mu);
    Variant &var = v.map[key];
    var.state = ok ? Variant::READY : Variant::FAILED;
    var.code.swap(code);
    var.from_disk = disk;
    if (ok) (disk ? v.disk_hits : v.compiled) += 1;
    v.cv.notify_all();
    return ok;
}

}  // namespace ats
