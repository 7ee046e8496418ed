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
    if (mode == 0 || !variant_eligible(prog)) return false;
    const uint64_t key = variant_key(prog);
    hipFunction_t fn = nullptr;
    {
        std::unique_lock<std::mutex> lk(v.mu);
        auto it = v.map.find(key);
        if (it == v.map.end()) {
            if ((int64_t)v.map.size() >= kMaxVariants) return false;
            const std::string src = generate(prog);
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
                hipModuleGetFunction(&f, mod, "atsv") != hipSuccess) {
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

bool variant_prepare(const MicroProg &prog, std::string &src) {
    if (!variant_eligible(prog)) return false;
    src = generate(prog);
    const uint64_t key = variant_key(prog);
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
