// Per-graph generated sparse SB kernel.
//
// For a small sparse graph the fastest layout on CDNA is one replica per lane
// with every soft spin x_i, momentum y_i and folded edge coefficient in
// VGPRs: the graph (which x_j feeds which y_i) is fixed for the whole run, so
// it is emitted as straight-line code and the T-step loop touches no memory
// except one scalar load of the step coefficient.  A VGPR cannot be indexed by
// a run-time neighbour id without extra instructions, hence the code is
// generated per graph and compiled once, device-only, by the ROCm clang found
// at ROCM_PATH (child process), then loaded as a module on the problem's
// device.  The instance's integer weights are baked in as literals for the
// fused exact cut evaluation.  The noise-injected variant (Eq. 10) draws the
// same counter-based Gaussian stream as the generic kernel, with the same
// float operations, and links the ROCm device library for cosine.
#include <dirent.h>
#include <fcntl.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <cctype>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <set>
#include <sstream>

#include "internal.hpp"

extern char **environ;

namespace qaia {

struct JitKernel {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    int device = 0;
};

void jit_release(JitKernel *k) {
    if (!k) return;
    if (k->mod) {
        DeviceGuard g(k->device);
        (void)hipModuleUnload(k->mod);
    }
    delete k;
}

bool jit_eligible(const Problem &p, std::string *why) {
    if (std::getenv("QAIA_DISABLE_JIT")) {
        if (why) *why = "disabled by QAIA_DISABLE_JIT";
        return false;
    }
    if (p.m > 8) {
        if (why) *why = "more than 8 objectives";
        return false;
    }
    // x, y and the edge coefficients live in VGPRs (plus ~20 temporaries);
    // keep the kernel within 256 VGPRs (two waves per SIMD).
    if (2 * (int64_t)p.n + p.E > 232) {
        if (why) *why = "graph too large for register-resident state";
        return false;
    }
    return true;
}

static const char *kPrelude = R"(#define __global__ __attribute__((global))
#define __device__ __attribute__((device))
#define __forceinline__ inline __attribute__((always_inline))
typedef unsigned long long u64;
typedef long long i64;
typedef unsigned int u32;
__device__ __forceinline__ u64 sm64(u64 seed, u64 idx) {
  u64 z = seed + (idx + 1ull) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ float initv(u64 seed, u64 idx, float amp) {
  u64 b = sm64(seed, idx);
  float u = (float)(u32)(b >> 40) * 0x1p-24f;
  return amp * (2.0f * u - 1.0f);
}
)";

// Box-Muller on two 24-bit uniforms of one draw from the noise-keyed stream.
static const char *kNoisePrelude = R"(extern "C" __device__ float __ocml_cos_f32(float);
__device__ __forceinline__ float nzv(u64 seed, u64 idx) {
  u64 b = sm64(seed ^ 0xd1b54a32d192ed03ull, idx);
  float u1 = (float)((u32)(b >> 40) + 1u) * 0x1p-24f;
  float u2 = (float)(u32)(b & 0xffffffull) * 0x1p-24f;
  return __builtin_sqrtf(-2.0f * __builtin_logf(u1)) * __ocml_cos_f32(6.2831853071795864769f * u2);
}
)";

// Register budget of a generated kernel: the compiler is asked for at least
// `waves` waves per SIMD (512 / waves VGPRs per lane).
static std::string waves_attr(int waves) {
    return ", amdgpu_waves_per_eu(" + std::to_string(waves) + ")";
}

static std::string generate(const Problem &p, int variant, bool trace, bool noise, int waves, bool pair_wall) {
    const int n = p.n, m = p.m;
    const int64_t E = p.E;
    const bool dsb = variant == QAIA_DSB;
    std::ostringstream s;
    s << kPrelude;
    if (noise) s << kNoisePrelude;
    s << "extern \"C\" __global__ __attribute__((amdgpu_flat_work_group_size(1, 256)" << waves_attr(waves) << "))\n"
         "void qaia_sb_reg(const float* __restrict__ jcp, const double* __restrict__ c0s,\n"
         "  const float* __restrict__ kt_tab, i64 rows, int R, int T, float dta0, u64 seed,\n"
         "  u64 offset, float amp, u64* __restrict__ spins, i64* __restrict__ obj,\n"
         "  float* __restrict__ trace, int trace_steps, float dt_alpha) {\n";
    s << "  const i64 row = (i64)__builtin_amdgcn_workgroup_id_x() * 256 + "
         "(i64)__builtin_amdgcn_workitem_id_x();\n";
    s << "  if (row >= rows) return;\n";
    s << "  const i64 w = row / R;\n";
    s << "  const u64 g = (u64)row + offset;\n";
    s << "  if (c0s[w] < 0.0) {\n";
    for (int wd = 0; wd < p.words; ++wd) s << "    spins[row * " << p.words << " + " << wd << "] = 0ull;\n";
    for (int k = 0; k < m; ++k) s << "    obj[row * " << m << " + " << k << "] = 0ll;\n";
    s << "    return;\n  }\n";
    // "+ 0.0f" turns a -0 start (init_amp = 0) into +0, so x is never -0 and
    // sgn(x) = copysign(1, x) agrees with sgn(0) = +1
    // an empty asm after each spin's start values keeps the compiler from
    // interleaving all 2n 64-bit hash computations, which pushed the prologue
    // past the register budget and spilled to scratch
    for (int i = 0; i < n; ++i)
        s << "  float X" << i << " = initv(seed, ((g * " << n << "ull + " << i << "ull) << 1), amp) + 0.0f, Y"
          << i << " = initv(seed, ((g * " << n << "ull + " << i << "ull) << 1) | 1ull, amp);\n"
          << "  asm volatile(\"\" : \"+v\"(X" << i << "), \"+v\"(Y" << i << "));\n";
    s << "  const float* jr = jcp + w * " << E << "ll;\n";
    for (int64_t e = 0; e < E; ++e) s << "  const float J" << e << " = jr[" << e << "];\n";
    // The step coefficient and dt a0 are copied into VGPRs (an opaque move,
    // which the compiler cannot fold back into scalar operands): with the
    // FMAs reading them from scalar registers dSB ran 10 % slower on the
    // 42-node graph (bSB the same), as if such FMAs issued alone.
    s << "  float dtv; asm(\"v_mov_b32 %0, %1\" : \"=v\"(dtv) : \"s\"(dta0));\n";
    // One SB step at time index t.
    auto step = [&](const std::string &tv) {
        s << "    { const int t = " << tv << ";\n";
        s << "    const float kts = kt_tab[t]; float kt; asm(\"v_mov_b32 %0, %1\" : \"=v\"(kt) : \"s\"(kts));\n";
        if (noise) s << "    const u64 nb = (g * (u64)T + (u64)t) * " << n << "ull;\n";
        if (dsb)
            for (int i = 0; i < n; ++i)
                s << "    const float S" << i << " = __builtin_copysignf(1.0f, X" << i << ");\n";
        // y_i += kt x_i + sum_j Jc'_ij phi(x_j), every phi from the pre-step x
        for (int i = 0; i < n; ++i) {
            s << "    Y" << i << " = __builtin_fmaf(kt, X" << i << ", Y" << i << ");";
            for (int q = p.rowptr[i]; q < p.rowptr[i + 1]; ++q)
                s << " Y" << i << " = __builtin_fmaf(J" << p.eid[q] << ", " << (dsb ? "S" : "X") << p.col[q] << ", Y"
                  << i << ");";
            if (noise) s << " Y" << i << " = __builtin_fmaf(dt_alpha, nzv(seed, nb + " << i << "ull), Y" << i << ");";
            s << "\n";
        }
        // x_i += dt a0 y_i, then the inelastic wall: |x| > 1 zeroes y, clamps x.
        // pair_wall writes the test as "clamping changed x", the same for every
        // finite x (and -0 == +0): a compare of two registers has the 32-bit
        // encoding, which the SIMD can issue together with another wave's
        // instruction, where |x| > 1 needs the 64-bit encoding (for the abs
        // modifier) and issues alone.
        for (int i = 0; i < n; ++i) {
            s << "    X" << i << " = __builtin_fmaf(dtv, Y" << i << ", X" << i << ");";
            if (pair_wall)
                s << " { const float C = __builtin_fminf(__builtin_fmaxf(X" << i << ", -1.0f), 1.0f); Y" << i
                  << " = C != X" << i << " ? 0.0f : Y" << i << "; X" << i << " = C; }\n";
            else
                s << " Y" << i << " = __builtin_fabsf(X" << i << ") > 1.0f ? 0.0f : Y" << i << "; X" << i
                  << " = __builtin_fminf(__builtin_fmaxf(X" << i << ", -1.0f), 1.0f);\n";
        }
        if (trace) {  // test hook only: the plain kernel carries no trace code
            s << "    if (t < trace_steps) {\n";
            s << "      float* tr = trace + (row * trace_steps + t) * " << n << "ll;\n";
            for (int i = 0; i < n; ++i) s << "      tr[" << i << "] = X" << i << ";\n";
            s << "    }\n";
        }
        s << "    }\n";
    };
    if (pair_wall) {
        // two steps per loop iteration: the clamped and the unclamped x are
        // both live at the wall test, and alternating their registers between
        // the two copies of the step leaves no copy at the back edge; the
        // scheduling barrier keeps the copies apart, so that the live values
        // stay those of one step (interleaved, dSB's spilled)
        s << "  int t0 = 0;\n  for (; t0 + 1 < T; t0 += 2) {\n";
        step("t0");
        s << "    __builtin_amdgcn_sched_barrier(0);\n";
        step("t0 + 1");
        s << "  }\n  if (t0 < T) {\n";
        step("t0");
        s << "  }\n";
    } else {
        s << "  for (int t0 = 0; t0 < T; ++t0) {\n";
        step("t0");
        s << "  }\n";
    }
    // read-out: bit i set <=> x_i < 0 (sgn 0 = +1)
    for (int wd = 0; wd < p.words; ++wd) {
        s << "  { u64 b = 0ull;";
        for (int i = wd * 64; i < n && i < wd * 64 + 64; ++i)
            s << " b |= (u64)(X" << i << " < 0.0f) << " << (i - wd * 64) << ";";
        s << " spins[row * " << p.words << " + " << wd << "] = b; }\n";
    }
    // exact cut values, Eq. (1), weights as literals
    for (int k = 0; k < m; ++k) {
        int64_t absum = 0;
        for (int64_t e = 0; e < E; ++e) absum += std::llabs((long long)p.W[(size_t)k * E + e]);
        const bool narrow = absum < (int64_t(1) << 31);
        s << "  { " << (narrow ? "int" : "i64") << " a = 0;";
        for (int64_t e = 0; e < E; ++e) {
            const int32_t wv = p.W[(size_t)k * E + e];
            if (wv == 0) continue;
            s << " a += ((X" << p.eu[e] << " < 0.0f) != (X" << p.ev[e] << " < 0.0f)) ? ("
              << (narrow ? "int" : "i64") << ")(" << wv << ") : 0;";
        }
        s << " obj[row * " << m << " + " << k << "] = (i64)a; }\n";
    }
    s << "}\n";
    return s.str();
}

// Half-precision form (QAIA_FP16): each lane carries two replicas (rows
// 2l and 2l + 1) as packed binary16 pairs, so every update is one packed
// fused multiply-add for both.  x and y start as the float32 draws rounded to
// binary16; the folded edge coefficients (per replica: the two rows may
// belong to different weight vectors), the step coefficient, dt a0 and
// dt alpha are the float32 values of the single-precision form rounded to
// binary16; the noise draw is computed in float32 and rounded.  Read-out and
// cut evaluation are exact, per replica.
static std::string generate16(const Problem &p, int variant, bool trace, bool noise, int waves) {
    const int n = p.n, m = p.m;
    const int64_t E = p.E;
    const bool dsb = variant == QAIA_DSB;
    std::ostringstream s;
    s << kPrelude;
    if (noise) s << kNoisePrelude;
    s << "typedef _Float16 h2 __attribute__((ext_vector_type(2)));\n"
         "__device__ __forceinline__ h2 hp(float a, float b) { h2 r; r.x = (_Float16)a; r.y = (_Float16)b; return r; }\n"
         "__device__ __forceinline__ h2 fm(h2 a, h2 b, h2 c) { return __builtin_elementwise_fma(a, b, c); }\n";
    s << "extern \"C\" __global__ __attribute__((amdgpu_flat_work_group_size(1, 256)" << waves_attr(waves) << "))\n"
         "void qaia_sb_reg(const float* __restrict__ jcp, const double* __restrict__ c0s,\n"
         "  const float* __restrict__ kt_tab, i64 rows, int R, int T, float dta0, u64 seed,\n"
         "  u64 offset, float amp, u64* __restrict__ spins, i64* __restrict__ obj,\n"
         "  float* __restrict__ trace, int trace_steps, float dt_alpha) {\n";
    s << "  const i64 pr = (i64)__builtin_amdgcn_workgroup_id_x() * 256 + (i64)__builtin_amdgcn_workitem_id_x();\n";
    // "+ zero" turns a -0 start into +0 (sgn 0 = +1 through copysign)
    s << "  const h2 one = hp(1.0f, 1.0f), zero = hp(0.0f, 0.0f);\n";
    s << "  const i64 r0 = pr * 2, r1 = r0 + 1;\n";
    s << "  if (r0 >= rows) return;\n";
    s << "  const bool has1 = r1 < rows;\n";
    s << "  const i64 w0 = r0 / R, w1 = has1 ? r1 / R : w0;\n";
    s << "  const u64 g0 = (u64)r0 + offset, g1 = (u64)r1 + offset;\n";
    s << "  const bool ok0 = c0s[w0] >= 0.0, ok1 = has1 && c0s[w1] >= 0.0;\n";
    for (int i = 0; i < n; ++i)
        s << "  h2 X" << i << " = hp(initv(seed, ((g0 * " << n << "ull + " << i << "ull) << 1), amp), initv(seed, ((g1 * "
          << n << "ull + " << i << "ull) << 1), amp)) + zero, Y" << i << " = hp(initv(seed, ((g0 * " << n
          << "ull + " << i << "ull) << 1) | 1ull, amp), initv(seed, ((g1 * " << n << "ull + " << i
          << "ull) << 1) | 1ull, amp));\n"
          << "  asm volatile(\"\" : \"+v\"(X" << i << "), \"+v\"(Y" << i << "));\n";
    s << "  const float* ja = jcp + w0 * " << E << "ll;\n";
    s << "  const float* jb = jcp + w1 * " << E << "ll;\n";
    for (int64_t e = 0; e < E; ++e) s << "  const h2 J" << e << " = hp(ja[" << e << "], jb[" << e << "]);\n";
    s << "  const h2 dA = hp(dta0, dta0), mB = hp(-1024.0f, -1024.0f), pB = hp(1025.0f, 1025.0f);\n";
    if (noise) s << "  const h2 dN = hp(dt_alpha, dt_alpha);\n";
    s << "  for (int t = 0; t < T; ++t) {\n";
    s << "    const h2 kt = hp(kt_tab[t], kt_tab[t]);\n";
    if (noise) {
        s << "    const u64 na = (g0 * (u64)T + (u64)t) * " << n << "ull;\n";
        s << "    const u64 nb = (g1 * (u64)T + (u64)t) * " << n << "ull;\n";
    }
    if (dsb)
        for (int i = 0; i < n; ++i)
            s << "    const h2 S" << i << " = __builtin_elementwise_copysign(one, X" << i << ");\n";
    for (int i = 0; i < n; ++i) {
        s << "    Y" << i << " = fm(kt, X" << i << ", Y" << i << ");";
        for (int q = p.rowptr[i]; q < p.rowptr[i + 1]; ++q)
            s << " Y" << i << " = fm(J" << p.eid[q] << ", " << (dsb ? "S" : "X") << p.col[q] << ", Y" << i << ");";
        if (noise)
            s << " Y" << i << " = fm(dN, hp(nzv(seed, na + " << i << "ull), nzv(seed, nb + " << i << "ull)), Y" << i
              << ");";
        s << "\n";
    }
    // the wall without per-half compares: with a = |x| (sign bits cleared),
    // f = min(max(1025 - 1024 a, 0), 1) is 1 for a <= 1 and 0 for a > 1
    // (the binary16 values above 1 start at 1 + 2^-10, where 1025 - 1024 a = 0;
    // the fused form rounds once and monotonically, so no value crosses), and
    // y * f zeroes y exactly where the wall hits
    for (int i = 0; i < n; ++i) {
        s << "    X" << i << " = fm(dA, Y" << i << ", X" << i << "); Y" << i
          << " = Y" << i << " * __builtin_elementwise_min(__builtin_elementwise_max(fm(__builtin_bit_cast(h2, "
             "__builtin_bit_cast(u32, X" << i << ") & 0x7fff7fffu), mB, pB), zero), one); X" << i
          << " = __builtin_elementwise_min(__builtin_elementwise_max(X" << i << ", -one), one);\n";
    }
    if (trace) {
        s << "    if (t < trace_steps) {\n";
        s << "      float* t0 = trace + (r0 * trace_steps + t) * " << n << "ll;\n";
        s << "      float* t1 = trace + (r1 * trace_steps + t) * " << n << "ll;\n";
        for (int i = 0; i < n; ++i)
            s << "      t0[" << i << "] = (float)X" << i << ".x; if (has1) t1[" << i << "] = (float)X" << i << ".y;\n";
        s << "    }\n";
    }
    s << "  }\n";
    for (int half = 0; half < 2; ++half) {
        const char *row = half ? "r1" : "r0";
        const char *ok = half ? "ok1" : "ok0";
        const char *c = half ? ".y" : ".x";
        s << "  if (" << (half ? "has1" : "true") << ") {\n";
        for (int wd = 0; wd < p.words; ++wd) {
            s << "    { u64 b = 0ull;";
            for (int i = wd * 64; i < n && i < wd * 64 + 64; ++i)
                s << " b |= (u64)(X" << i << c << " < (_Float16)0.0f) << " << (i - wd * 64) << ";";
            s << " spins[" << row << " * " << p.words << " + " << wd << "] = " << ok << " ? b : 0ull; }\n";
        }
        for (int k = 0; k < m; ++k) {
            int64_t absum = 0;
            for (int64_t e = 0; e < E; ++e) absum += std::llabs((long long)p.W[(size_t)k * E + e]);
            const bool narrow = absum < (int64_t(1) << 31);
            s << "    { " << (narrow ? "int" : "i64") << " a = 0;";
            for (int64_t e = 0; e < E; ++e) {
                const int32_t wv = p.W[(size_t)k * E + e];
                if (wv == 0) continue;
                s << " a += ((X" << p.eu[e] << c << " < (_Float16)0.0f) != (X" << p.ev[e] << c
                  << " < (_Float16)0.0f)) ? (" << (narrow ? "int" : "i64") << ")(" << wv << ") : 0;";
            }
            s << " obj[" << row << " * " << m << " + " << k << "] = " << ok << " ? (i64)a : 0ll; }\n";
        }
        s << "  }\n";
    }
    s << "}\n";
    return s.str();
}

static uint64_t fnv1a(const std::string &s) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 0x100000001b3ull;
    }
    return h;
}

static std::string rocm_root() {
    if (const char *r = std::getenv("ROCM_PATH")) return r;
    return "/opt/rocm";
}

static std::string find_clang() {
    if (const char *e = std::getenv("QAIA_CLANG")) return e;
    return rocm_root() + "/llvm/bin/clang++";
}

// Compile one source to a raw gfx950 code object in a private temp dir;
// device_libs links the ROCm device library (needed by the noise variant);
// listing, when given, receives the compiler's assembly of the kernel.
static std::vector<char> compile(const std::string &src, bool device_libs, std::string *listing = nullptr) {
    const char *tmpenv = std::getenv("TMPDIR");
    std::string tmpl = std::string(tmpenv && *tmpenv ? tmpenv : "/tmp") + "/qaia_jit_XXXXXX";
    std::vector<char> dirbuf(tmpl.begin(), tmpl.end());
    dirbuf.push_back('\0');
    QAIA_CHECK(mkdtemp(dirbuf.data()) != nullptr, QAIA_UNSUPPORTED,
               "cannot create a temporary directory for kernel generation");
    const std::string dir(dirbuf.data());
    const std::string in = dir + "/k.hip", out = dir + "/k.hsaco", log = dir + "/k.log";
    {
        std::ofstream f(in);
        f << src;
    }
    const std::string clang = find_clang();
    std::vector<std::string> args = {clang,
                                     "-x",
                                     "hip",
                                     "--offload-arch=gfx950",
                                     "--offload-device-only",
                                     "--no-gpu-bundle-output",
                                     "-nogpuinc",
                                     device_libs ? "--rocm-path=" + rocm_root() : std::string("-nogpulib"),
                                     "-O3",
                                     "-mcode-object-version=5",
                                     "-Xclang",
                                     "-target-feature",
                                     "-Xclang",
                                     "-packed-fp32-ops",
                                     "-c",
                                     in,
                                     "-o",
                                     out};
    if (listing) args.push_back("-save-temps=obj");  // intermediates, the .s among them, beside out
    std::vector<char *> argv;
    for (auto &a : args) argv.push_back(const_cast<char *>(a.c_str()));
    argv.push_back(nullptr);
    posix_spawn_file_actions_t fa;
    posix_spawn_file_actions_init(&fa);
    posix_spawn_file_actions_addopen(&fa, 1, log.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0600);
    posix_spawn_file_actions_adddup2(&fa, 1, 2);
    pid_t pid;
    int rc = posix_spawn(&pid, clang.c_str(), &fa, nullptr, argv.data(), environ);
    posix_spawn_file_actions_destroy(&fa);
    std::vector<char> code;
    std::string err;
    if (rc != 0) {
        err = "cannot start " + clang + ": " + std::strerror(rc);
    } else {
        int status = 0;
        pid_t w;
        do {  // a signal may interrupt the wait before the compiler exits
            w = waitpid(pid, &status, 0);
        } while (w < 0 && errno == EINTR);
        if (w < 0) {
            err = std::string("waiting for the kernel compiler failed: ") + std::strerror(errno);
        } else if (!WIFEXITED(status) || WEXITSTATUS(status) != 0) {
            std::ifstream lf(log);
            std::stringstream ls;
            ls << lf.rdbuf();
            err = "kernel generation failed: " + ls.str().substr(0, 2000);
        } else {
            std::ifstream f(out, std::ios::binary);
            code.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
            if (code.empty()) err = "kernel generation produced no code object";
            if (listing) {
                std::ifstream sf(dir + "/k-hip-amdgcn-amd-amdhsa-gfx950.s");
                std::stringstream ss;
                ss << sf.rdbuf();
                *listing = ss.str();
            }
        }
    }
    // the directory holds only what this call created
    if (DIR *d = opendir(dir.c_str())) {
        while (dirent *ent = readdir(d)) {
            const std::string name = ent->d_name;
            if (name != "." && name != "..") std::remove((dir + "/" + name).c_str());
        }
        closedir(d);
    }
    rmdir(dir.c_str());
    QAIA_CHECK(err.empty(), QAIA_UNSUPPORTED, err);
    return code;
}

// True when the listing shows spill traffic (scratch or buffer accesses,
// accumulation-register copies) inside an outermost loop, i.e. between a
// loop header's label and the first branch back to it.
static bool loop_spills(const std::string &s) {
    const std::string mark = "Loop Header: Depth=1";
    for (size_t h = s.find(mark); h != std::string::npos; h = s.find(mark, h + 1)) {
        const size_t ls = s.rfind('\n', h) + 1;  // npos + 1 == 0 at the first line
        const size_t colon = s.find(':', ls);
        if (colon == std::string::npos || colon > h) continue;
        const std::string label = s.substr(ls, colon - ls);
        size_t end = std::string::npos;
        for (size_t q = s.find(label, h); q != std::string::npos; q = s.find(label, q + 1)) {
            const size_t after = q + label.size();
            if (after < s.size() && std::isalnum((unsigned char)s[after])) continue;  // .LBB0_8 vs .LBB0_80
            const size_t line = s.rfind('\n', q) + 1;
            if (s.compare(line, 1, "\t") == 0 && s.find("branch", line) < q) {
                end = q;
                break;
            }
        }
        if (end == std::string::npos) continue;
        const std::string body = s.substr(h, end - h);
        if (body.find("scratch_") != std::string::npos || body.find("buffer_") != std::string::npos ||
            body.find("accvgpr") != std::string::npos)
            return true;
    }
    return false;
}

static std::mutex g_cache_mu;
static std::map<uint64_t, std::vector<char>> g_cache;  // source hash -> code object
static std::set<uint64_t> g_spilling;                  // sources whose step loop spills

// Build candidates in order of preference, (waves per SIMD, paired wall
// test): the first whose step loop the compiler keeps free of spill traffic
// is taken, the last one regardless.  Three waves per SIMD (168 VGPRs) give
// each issue slot more candidates than two (5-7 % on the 42-node graph); two
// (256 VGPRs) keep every graph the path admits in registers.  The paired
// wall test saves an issue slot per spin and step (about 8 % for bSB on the
// 42-node graph); it is not tried with the noise generator, whose registers
// leave no room for it.  The
// binary16 kernels always ask for two waves: their packed instructions issue
// one per slot whatever the occupancy, and three measured 1-4 % slower.
// (Loading the edge coefficients once per wave into scalar registers,
// possible when R is a multiple of 64, frees their VGPRs but made both
// variants a third slower at every occupancy from two to four waves.)
static JitKernel *build_kernel(const Problem &p, int variant, bool trace, bool noise, bool half = false) {
    struct Candidate {
        int waves;
        bool pair_wall;
    };
    std::vector<Candidate> cands;
    if (half) {
        cands = {{2, false}};
    } else {
        const bool pair = !noise;
        // three waves leave 168 VGPRs: past 160 state registers (2n + E) every
        // build spilled
        for (int waves = 2 * (int64_t)p.n + p.E <= 160 ? 3 : 2; waves >= 2; --waves) {
            if (pair) cands.push_back({waves, true});
            cands.push_back({waves, false});
        }
    }
    std::vector<char> code;
    for (size_t ci = 0; ci < cands.size() && code.empty(); ++ci) {
        const bool last = ci + 1 == cands.size();
        const Candidate cd = cands[ci];
        const std::string src = half ? generate16(p, variant, trace, noise, cd.waves)
                                     : generate(p, variant, trace, noise, cd.waves, cd.pair_wall);
        const uint64_t h = fnv1a(src);
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            if (g_spilling.count(h)) continue;
            auto it = g_cache.find(h);
            if (it != g_cache.end()) code = it->second;
        }
        if (!code.empty()) break;
        std::string listing;
        std::vector<char> c = compile(src, noise, last ? nullptr : &listing);
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (!last && (listing.empty() || loop_spills(listing))) {
            g_spilling.insert(h);
            continue;
        }
        g_cache[h] = c;
        code.swap(c);
    }
    JitKernel *k = new JitKernel();
    k->device = p.device;
    DeviceGuard g(p.device);
    hipError_t e = hipModuleLoadData(&k->mod, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&k->fn, k->mod, "qaia_sb_reg");
    if (e != hipSuccess) {
        std::string msg = std::string("loading the generated kernel: ") + hipGetErrorString(e);
        jit_release(k);
        throw Error{QAIA_DEVICE_ERROR, msg};
    }
    return k;
}

void jit_prepare(Problem &p) {
    std::string why;
    if (!jit_eligible(p, &why)) {
        p.jit_error = why;
        return;
    }
    for (int variant = 0; variant < 2; ++variant) {
        try {
            p.jit[variant] = build_kernel(p, variant, false, false);
        } catch (const Error &err) {
            p.jit_error = err.msg;
            return;
        }
    }
}

// The tracing variants (trajectory tests) and the noise-injected variants are
// generated on first use.
// The binary16 variants too.
static const JitKernel *kernel_for(const Problem &p, int variant, bool trace, bool noise, bool half) {
    if (!trace && !noise && !half) return p.jit[variant];
    Problem &mp = const_cast<Problem &>(p);
    std::lock_guard<std::mutex> lk(mp.mu);
    JitKernel *&slot = half ? mp.jit16[variant][trace ? 1 : 0][noise ? 1 : 0]
                            : noise ? mp.jit_noise[variant][trace ? 1 : 0] : mp.jit_trace[variant];
    if (!slot) slot = build_kernel(p, variant, trace, noise, half);
    return slot;
}

bool sparse_reg_ready(const Problem &p, int variant, bool trace, bool noise, bool half) {
    if (!trace && !noise && !half) return p.jit[variant] != nullptr;
    Problem &mp = const_cast<Problem &>(p);
    std::lock_guard<std::mutex> lk(mp.mu);
    return (half ? mp.jit16[variant][trace ? 1 : 0][noise ? 1 : 0]
                 : noise ? mp.jit_noise[variant][trace ? 1 : 0] : mp.jit_trace[variant]) != nullptr;
}

void launch_sparse_reg(const Problem &p, int variant, int64_t W, int32_t R, const qaia_schedule &s,
                       void *ws, const WsLayout &L, uint64_t *spins, int64_t *obj, float *trace,
                       int32_t trace_steps, hipStream_t st) {
    QAIA_CHECK(p.jit[variant] != nullptr, QAIA_UNSUPPORTED,
               "register-resident path unavailable: " + (p.jit_error.empty() ? std::string("not built") : p.jit_error));
    float dt_alpha = s.dt * s.noise_alpha;
    const bool half = s.precision == QAIA_FP16;
    const JitKernel *k = kernel_for(p, variant, trace != nullptr, dt_alpha != 0.0f, half);
    const int64_t rows = W * (int64_t)R;
    if (rows == 0) return;
    const int64_t lanes = half ? (rows + 1) / 2 : rows;  // binary16: two replicas per lane
    const int64_t blocks = (lanes + 255) / 256;
    QAIA_CHECK(blocks <= INT32_MAX, QAIA_INVALID_ARGUMENT, "too many replicas for one launch");
    char *b = (char *)ws;
    const float *jcp = (const float *)(b + L.jcp), *kt = (const float *)(b + L.kt);
    const double *c0s = (const double *)(b + L.c0s);
    int T = s.steps;
    float dta0 = s.dt * s.a0, amp = s.init_amp;
    uint64_t seed = s.seed, off = s.replica_offset;
    int64_t rows_ = rows;
    int R_ = R, ts = trace_steps;
    void *args[] = {(void *)&jcp, (void *)&c0s, (void *)&kt,   (void *)&rows_, (void *)&R_,
                    (void *)&T,   (void *)&dta0, (void *)&seed, (void *)&off,  (void *)&amp,
                    (void *)&spins, (void *)&obj, (void *)&trace, (void *)&ts, (void *)&dt_alpha};
    QAIA_HIP(hipModuleLaunchKernel(k->fn, (unsigned)blocks, 1, 1, 256, 1, 1, 0, st, args, nullptr));
}

}  // namespace qaia
