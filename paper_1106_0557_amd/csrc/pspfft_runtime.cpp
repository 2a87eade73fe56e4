// pspfft_runtime.cpp -- host side of the C ABI declared in include/pspfft.h:
// size validation, per-axis stage plans and twiddle tables, the resident
// Green's-function spectrum (computed once at plan creation, Sec. 2.2.2), default
// and caller workspaces, and grouped launches of the five passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <utility>
#include <numeric>
#include <vector>

#include "../../include/pspfft.h"
#include "internal.h"

using pspfft::AxisPlan;
using pspfft::DevPlan;
using pspfft::LaunchArgs;
using pspfft::ProbArg;

struct pspfft_plan_s {
    int n[3];
    double h[3];
    pspfft_precision prec;
    DevPlan host;            // copy of the device plan (device pointers inside)
    DevPlan *dev = nullptr;  // device copy read by the kernels
    void *tw[3] = {nullptr, nullptr, nullptr};
    void *G = nullptr, *Gn = nullptr;
    pspfft_workspace_t ws = nullptr;  // default workspace, allocated by the first pspfft_solve
    size_t bytes = 0;        // resident bytes (without the default workspace)
    int device = 0;
    bool fused = false;      // x and y transforms of a z plane in one kernel
    int pE = 0, pK = 0;      // radix family and last radix of those kernels
    int verbosity = -1;      // the plan's own message level (Sec. 3.2, VerbosityOption); -1: the process's
    std::mutex mu;           // guards the creation of the default workspace
};

struct pspfft_workspace_s {
    pspfft_plan_t plan;
    void *mem;
    bool owned;
    void *W;
    void *Wn;
    size_t bytes;
};

namespace {

// ------------------------------------------------------------------ messages --
// Levels of Sec. 3.2's VerbosityOption, least verbose first: errors (the
// default), warnings, then two levels of information.  The process level starts
// from PSPFFT_LOG (error | warn | info1 | info2) and is changed by
// pspfft_set_verbosity; a plan created with a verbosity option keeps its own.
// Messages go to stderr, or to the callback set with pspfft_set_log_callback.
std::atomic<int> g_level{-1};
std::mutex g_log_mu;
pspfft_log_fn g_log_fn = nullptr;
void *g_log_user = nullptr;

int process_level() {
    int l = g_level.load(std::memory_order_relaxed);
    if (l >= 0) return l;
    l = PSPFFT_CONSOLE_ERROR;
    if (const char *e = std::getenv("PSPFFT_LOG")) {
        if (!std::strcmp(e, "warn")) l = PSPFFT_CONSOLE_WARNING;
        else if (!std::strcmp(e, "info1")) l = PSPFFT_CONSOLE_INFO_1;
        else if (!std::strcmp(e, "info2")) l = PSPFFT_CONSOLE_INFO_2;
    }
    int unset = -1;
    g_level.compare_exchange_strong(unset, l);
    return g_level.load(std::memory_order_relaxed);
}

// Level in force for messages about a plan whose own level is `plan_level`.
int level_for(int plan_level) { return plan_level >= 0 ? plan_level : process_level(); }

void emit(int lvl, const char *fmt, ...) {
    char buf[640];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> lk(g_log_mu);
    if (g_log_fn) {
        g_log_fn(static_cast<pspfft_verbosity>(lvl), buf, g_log_user);
    } else {
        static const char *const tag[4] = {"error", "warning", "info", "info"};
        std::fprintf(stderr, "[pspfft %s] %s\n", tag[lvl & 3], buf);
    }
}

#define PSPFFT_MSG(plan_level, lvl, ...)                                        \
    do {                                                                        \
        if (level_for(plan_level) >= (lvl)) emit((lvl), __VA_ARGS__);          \
    } while (0)
#define PSPFFT_LOG(lvl, ...) PSPFFT_MSG(-1, lvl, __VA_ARGS__)

// Report a failed call (level error) and return its status.
pspfft_status fail(pspfft_status st, int plan_level, const char *fmt, ...) {
    if (level_for(plan_level) >= PSPFFT_CONSOLE_ERROR) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        emit(PSPFFT_CONSOLE_ERROR, "%s: %s", buf, pspfft_status_string(st));
    }
    return st;
}

// Workgroup renumbering for the XCDs, per pass (0 none, 1 contiguous eighths,
// 2 runs of 8 within blocks of 64).  PSPFFT_XCD_REMAP="abcde" overrides the
// five passes in order.  Measured: the row passes and the y passes gain from
// contiguous eighths (y passes of one solve: FP64 768^3 8.0 / 8.9 -> 6.8 /
// 7.0 ms, 256^3 0.156 / 0.160 -> 0.146 / 0.147 ms; FP32 1152^3, whose column
// kernel keeps its twiddles in global memory, 32.7 / 21.3 -> 14.1 / 12.4 ms),
// the z pass loses.
int xcd_remap_mode(int mode) {
    static int modes[5] = {-1, -1, -1, -1, -1};
    if (modes[0] < 0) {
        const int dflt[5] = {1, 1, 0, 1, 1};
        const char *e = std::getenv("PSPFFT_XCD_REMAP");
        for (int i = 0; i < 5; ++i) {
            int v = dflt[i];
            if (e && std::strlen(e) == 5 && e[i] >= '0' && e[i] <= '2') v = e[i] - '0';
            modes[i] = v;
        }
    }
    return (mode >= 0 && mode < 5) ? modes[mode] : 0;
}

// FP32 z lines of 2048 points on the 32-family (radices 32, 32, 2: 64 threads
// per line, so the line fits one wavefront; PSPFFT_Z32=0 keeps the 16-family's
// 16, 16, 8, 128 threads per line).  Measured, one 1024^3 solve: z pass 24.4 ->
// 18.2 ms.  Lines of 1024 points stay on the 16-family: as 32 x 32 (two lines
// per wavefront, eight wavefronts per CU instead of sixteen) the 512^3 z pass
// takes 1.56 ms instead of 1.43.
bool z32_enabled() {
    static int v = -1;
    if (v < 0) {
        const char *e = std::getenv("PSPFFT_Z32");
        v = e && std::atoi(e) == 0 ? 0 : 1;
    }
    return v == 1;
}

// Lines per workgroup of each pass; PSPFFT_TILE="a,b,c,d,e" overrides (powers of two).
int line_tile(int mode, int dflt) {
    static int v[5] = {-1, -1, -1, -1, -1};
    if (v[0] < 0) {
        for (int i = 0; i < 5; ++i) v[i] = 0;
        if (const char *e = std::getenv("PSPFFT_TILE")) {
            int i = 0;
            for (const char *q = e; *q && i < 5; ++i) {
                v[i] = std::atoi(q);
                while (*q && *q != ',') ++q;
                if (*q == ',') ++q;
            }
        }
    }
    const int o = (mode >= 0 && mode < 5) ? v[mode] : 0;
    return (o > 0 && (o & (o - 1)) == 0) ? o : dflt;
}

size_t real_size(pspfft_precision p) { return p == PSPFFT_FP32 ? 4 : 8; }
size_t cplx_size(pspfft_precision p) { return 2 * real_size(p); }
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Radix family of a transform length L: the odd part o of L selects E, the
// elements each thread owns (every stage radix divides E); L must be a multiple
// of E.  y and z transforms have L = 2n; the packed x transform has L = n.
int family_of_len(int L) {
    if (L < 1) return 0;
    int m = L;
    while (m % 2 == 0) m /= 2;
    int E = 0;
    if (m == 1) E = 16;
    else if (m == 3) E = 24;
    else if (m == 5) E = 20;
    else if (m == 9) E = 36;
    else return 0;
    if (L < E || L % E != 0) return 0;
    return E;
}

int axis_len(int axis, int n) { return axis == 0 ? n : 2 * n; }

// Largest mesh size of the radix-family kernels per precision (y and z; the
// packed x transform has length n, so x may be twice as long).
int max_n(pspfft_precision p) { return p == PSPFFT_FP32 ? 2048 : 1152; }

// Largest mesh size of the generic line kernel, any axis and precision: the
// doubled line of 2n <= 4096 points and its two LDS buffers fit one workgroup.
constexpr int kGenericMaxN = 2048;

// n = 2^a 3^b 5^c
bool smooth235(int n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

// The axis runs on a radix family's kernels (else on the generic line kernel).
bool family_axis(int axis, int n, pspfft_precision p) {
    const int lim = axis == 0 ? 2 * max_n(p) : max_n(p);
    return n >= 1 && n <= lim && family_of_len(axis_len(axis, n)) != 0;
}

bool size_ok(int axis, int n, pspfft_precision p) {
    return family_axis(axis, n, p) || (n >= 1 && n <= kGenericMaxN && smooth235(n));
}

bool sizes_ok(int nx, int ny, int nz, pspfft_precision p) {
    return size_ok(0, nx, p) && size_ok(1, ny, p) && size_ok(2, nz, p);
}

// cos and sin of 2 pi j / M in double precision, folded into [0, pi/4] first.
void turn(long j, long M, double &c, double &s) {
    j %= M;
    if (j < 0) j += M;
    long num = j, den = M;
    bool neg_s = false, neg_c = false, swap = false;
    if (2 * num > den) { num = den - num; neg_s = true; }
    if (4 * num > den) { num = den - 2 * num; den *= 2; neg_c = true; }
    if (8 * num > den) { num = den - 4 * num; den *= 4; swap = true; }
    const double x = 2.0 * M_PI * static_cast<double>(num) / static_cast<double>(den);
    c = std::cos(x);
    s = std::sin(x);
    if (swap) std::swap(c, s);
    if (neg_c) c = -c;
    if (neg_s) s = -s;
}

// Radices of the generic line kernel for a length L = 2^a 3^b 5^c, in stage
// order: the largest of its radices that divides what is left, each time
// (few stages: every stage is a round trip through LDS).
std::vector<int> generic_radices(int L) {
    static const int kRadices[] = {27, 25, 16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
    std::vector<int> r;
    int m = L;
    while (m > 1) {
        int pick = 0;
        for (int R : kRadices)
            if (m % R == 0) {
                pick = R;
                break;
            }
        if (!pick) return {};  // not 2^a 3^b 5^c
        r.push_back(pick);
        m /= pick;
    }
    return r;
}

// Stage plan and FP64 twiddles of one axis: a radix family's stages (every
// radix divides E) where the family kernels take the length, else the generic
// kernel's radices.
bool build_axis(int axis, int n, pspfft_precision prec, AxisPlan &ax, std::vector<std::complex<double>> &tw,
                int force_E = 0) {
    const int L = axis_len(axis, n);
    const int E = force_E ? force_E : (family_axis(axis, n, prec) ? family_of_len(L) : 0);
    if (force_E && L % force_E != 0) return false;
    if (!E && !(n <= kGenericMaxN && smooth235(n))) return false;
    std::memset(&ax, 0, sizeof(ax));
    ax.n = n;
    ax.L = L;
    ax.E = E;
    ax.NB = E ? L / E : 0;
    const std::vector<int> gen = E ? std::vector<int>() : generic_radices(L);
    if (!E && static_cast<int>(gen.size()) > pspfft::kMaxStages) return false;
    int rem = L, Ns = 1, s = 0;
    tw.clear();
    while (rem > 1) {
        if (s >= pspfft::kMaxStages) return false;
        const int R = E ? std::gcd(E, rem) : gen[s];
        if (R <= 1 || rem % R != 0) return false;
        ax.R[s] = R;
        ax.Ns[s] = Ns;
        ax.magic[s] = Ns > 1 ? static_cast<uint32_t>((uint64_t(1) << 32) / Ns + 1) : 0u;
        if (E && Ns > 1) {  // verify the family kernels' multiply-high division for every index used
            for (uint32_t b = 0; b < static_cast<uint32_t>(L); ++b) {
                const uint32_t q = static_cast<uint32_t>((uint64_t(b) * ax.magic[s]) >> 32);
                if (q != b / static_cast<uint32_t>(Ns)) return false;
            }
        }
        ax.twoff[s] = static_cast<int>(tw.size());
        for (int k = 0; k < Ns; ++k)
            for (int r = 1; r < R; ++r) {
                double c, sn;
                turn(-static_cast<long>(r) * k, static_cast<long>(Ns) * R, c, sn);
                tw.emplace_back(c, sn);
            }
        Ns *= R;
        rem /= R;
        ++s;
    }
    ax.nst = s;
    ax.ntw = static_cast<int>(tw.size());
    if (axis == 0) {  // split-step factors exp(-i pi k / n) of the packed real transform
        for (int k = 0; k < n; ++k) {
            double c, sn;
            turn(-static_cast<long>(k), 2L * n, c, sn);
            tw.emplace_back(c, sn);
        }
    }
    if (tw.empty()) tw.emplace_back(1.0, 0.0);
    return Ns == L;
}

// cos(pi j / n), j < 2n, for the even-extension transform of G.
std::vector<double> cos_table(int n) {
    std::vector<double> t(2 * n);
    for (int j = 0; j < 2 * n; ++j) {
        double c, s;
        turn(j, 2L * n, c, s);
        t[j] = c;
    }
    return t;
}

template <typename F>
struct Guard {
    F f;
    bool armed = true;
    ~Guard() {
        if (armed) f();
    }
};
template <typename F>
Guard<F> make_guard(F f) { return Guard<F>{f}; }

pspfft_status alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return PSPFFT_ERR_OUT_OF_MEMORY;
    }
    return PSPFFT_OK;
}

size_t ws_bytes(const int n[3], pspfft_precision prec) {
    const size_t c = cplx_size(prec);
    const size_t main = static_cast<size_t>(n[2]) * 2 * n[1] * n[0] * c;
    const size_t nyq = static_cast<size_t>(n[2]) * 2 * n[1] * c;
    return round_up(main, 256) + round_up(nyq, 256);
}

void ws_split(pspfft_workspace_t w, const int n[3], pspfft_precision prec) {
    const size_t c = cplx_size(prec);
    const size_t main = static_cast<size_t>(n[2]) * 2 * n[1] * n[0] * c;
    w->W = w->mem;
    w->Wn = static_cast<char *>(w->mem) + round_up(main, 256);
}

// Frees with hipFree, which in the HIP runtime waits for all work queued on the
// device first (measured: a hipFree issued while another stream runs returns
// when that stream's work is done), so a plan's memory is never released under
// a kernel that still reads it.
void destroy_plan(pspfft_plan_t p) {
    if (!p) return;
    if (p->ws) {
        if (p->ws->owned && p->ws->mem) (void)hipFree(p->ws->mem);
        delete p->ws;
    }
    for (auto &t : p->tw)
        if (t) (void)hipFree(t);
    if (p->G) (void)hipFree(p->G);
    if (p->Gn) (void)hipFree(p->Gn);
    if (p->dev) (void)hipFree(p->dev);
    delete p;
}

// Every device array of a solve (source, potential, workspace, spectrum) is
// addressable with unsigned 32-bit byte offsets.
// Launches whose workspaces together exceed the Infinity Cache stream their
// line data (LaunchArgs::nt).
bool streaming_launch(const pspfft_plan_t *plans, const std::vector<int> &idx, size_t c0, size_t c1) {
    size_t b = 0;
    for (size_t j = c0; j < c1; ++j) b += ws_bytes(plans[idx[j]]->n, plans[idx[j]]->prec);
    return b > pspfft::kStreamBytes;
}

bool arrays_below_4gb(pspfft_plan_t p) {
    const size_t lim = size_t(1) << 32;
    const size_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
    const size_t r = real_size(p->prec);
    return ws_bytes(p->n, p->prec) < lim && nx * ny * nz * r < lim && (nz + 1) * (ny + 1) * nx * r < lim;
}

// The z pass runs by wavefront-owned lines (wave_col_kernel) where its lines
// have three stages E, M, K with M*K = 32 or 64 threads, or 16 threads where the
// tile's rows take more than half the LDS (one workgroup per CU; measured, the
// smaller 16-thread tiles gain nothing over the column kernel), or four stages
// in FP32 (E, M, M, K with 32 or 64 threads), and the compile-time instance
// exists.  Arrays of 4 GB or more take its 64-bit form, which needs a z line's
// NB-position block (NB*2ny*nx values) below 4 GB.  Such plans keep the
// spectrum kz-fastest, and their z launches always take that kernel.
bool z_wave_lines(pspfft_plan_t p) {
    const AxisPlan &az = p->host.ax[2];
    if (az.E == 0) return false;  // generic kernel
    const int prec = p->host.prec, M = az.E & -az.E, NB = az.NB;
    const size_t block_bytes = static_cast<size_t>(NB) * 2 * p->n[1] * p->n[0] * (prec == 0 ? 8 : 16);
    if (!arrays_below_4gb(p) && block_bytes >= (size_t(1) << 32) - 64) return false;
    if (az.nst == 4)  // four-stage FP32 lines of 32 or 64 threads, wave_tile() lines per workgroup
        return prec == 0 && M < az.E && az.R[1] == M && az.R[2] == M && M * M * az.R[3] == NB &&
               (NB == 32 || NB == 64) &&
               pspfft::wave_tile(prec, pspfft::Z_CONV, az.E, NB, 4) * NB <= pspfft::max_block_for(prec, az.E) &&
               pspfft::wave_lds_bytes(prec, pspfft::Z_CONV, az.E, NB, 4) <= 160 * 1024;
    const bool nb_ok = NB == 32 || NB == 64 || (NB == 16 && pspfft::wave_z_lds_bytes(prec, az.E, NB) > 80 * 1024);
    return az.nst == 3 && az.R[1] == M && nb_ok && M * az.R[2] == NB &&
           pspfft::wave_tile(prec, pspfft::Z_CONV, az.E, NB) * NB <= pspfft::max_block_for(prec, az.E) &&
           pspfft::wave_lds_bytes(prec, pspfft::Z_CONV, az.E, NB) <= 160 * 1024 &&
           pspfft::pass_tile(prec, pspfft::Y_FWD, az.E, NB) * NB <= pspfft::max_block_for(prec, az.E);
}

// Lines (main, Nyquist) that a pass processes for one problem.
void pass_lines(int mode, const int n[3], long &main, long &nyq) {
    const long nx = n[0], ny = n[1], nz = n[2];
    switch (mode) {
        case pspfft::X_FWD:
        case pspfft::X_INV: main = ny * nz; nyq = 0; break;
        case pspfft::Y_FWD:
        case pspfft::Y_INV: main = nz * nx; nyq = nz; break;
        default: main = 2 * ny * nx; nyq = 2 * ny; break;
    }
}

// Lines per workgroup of the generic kernel for lines of up to L points: the
// largest power of two up to 64 whose two LDS buffers fit 160 KB, with at most
// max(2L, 2048) points per workgroup (about 8 per thread, two lines at least).
// Its stage twiddles go into LDS too where they fit beside the buffers.
// Measured (one solve, FP32): at most 2048 points instead of 4096 (more
// workgroups per CU; with the chunked XCD order the narrower column tiles
// still meet in L2) takes 480^3 from 13.5 to 12.4 ms and FP64 480^3 from 26.8
// to 22.4 ms, but single-line tiles lose (960^3 y and z passes 17.0 / 66.4 ->
// 21.0 / 80.4 ms), hence two lines at least.
int generic_tile(int L, size_t csz) {
    int t = 64;
    while (t > 1 && (static_cast<size_t>(2) * t * (L + 1) * csz > 160 * 1024 ||
                     static_cast<long>(t) * L > std::max(2L * L, 2048L)))
        t /= 2;
    return t;
}

// Grouped launches of a pass on the generic line kernel: one per precision (and
// per kMaxProblems problems).  The launch's tile follows its longest line; a
// line's arithmetic does not depend on the tile (each butterfly reads only its
// own line), so results are the same alone and in any batch.
pspfft_status launch_generic_lines(int mode, const std::vector<int> &all, const pspfft_plan_t *plans,
                                   const pspfft_workspace_t *ws, const void *const *S, void *const *Phi,
                                   hipStream_t stream) {
    const int axis = pspfft::pass_axis(mode);
    std::map<int, std::vector<int>> groups;
    for (int i : all) groups[static_cast<int>(plans[i]->prec)].push_back(i);
    for (auto &kv : groups) {
        const int prec = kv.first;
        const size_t csz = prec == 0 ? 8 : 16;
        std::vector<int> idx = kv.second;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            return reinterpret_cast<uintptr_t>(plans[a]) < reinterpret_cast<uintptr_t>(plans[b]);
        });
        for (size_t c0 = 0; c0 < idx.size(); c0 += pspfft::kMaxProblems) {
            const size_t c1 = std::min(idx.size(), c0 + pspfft::kMaxProblems);
            LaunchArgs args;
            std::memset(&args, 0, sizeof(args));
            args.count = static_cast<int>(c1 - c0);
            int lmax = 1;
            for (size_t j = c0; j < c1; ++j) lmax = std::max(lmax, plans[idx[j]]->host.ax[axis].L);
            for (size_t j = c0; j < c1; ++j) {
                const int i = idx[j];
                ProbArg &a = args.p[j - c0];
                a.plan = plans[i]->dev;
                a.S = S ? S[i] : nullptr;
                a.Phi = Phi ? Phi[i] : nullptr;
                a.W = ws[i]->W;
                a.Wn = ws[i]->Wn;
                if (j > c0 && plans[idx[j - 1]] == plans[i]) {
                    args.seg[args.nseg - 1].group += 1;
                    continue;
                }
                pspfft::Segment &sg = args.seg[args.nseg++];
                sg.first = static_cast<int>(j - c0);
                sg.group = 1;
            }
            args.gtile = generic_tile(lmax, csz);
            args.glmax = lmax;
            int ntw = 0;
            for (size_t j = c0; j < c1; ++j) ntw = std::max(ntw, plans[idx[j]]->host.ax[axis].ntw);
            const size_t bufs = static_cast<size_t>(2) * args.gtile * (lmax + 1) * csz;
            args.gtw = bufs + ntw * csz <= 160 * 1024 ? 1 : 0;
            long wg = 0;
            for (int k = 0; k < args.nseg; ++k) {
                pspfft::Segment &sg = args.seg[k];
                const pspfft_plan_t pl = plans[idx[c0 + sg.first]];
                long lm, ln;
                pass_lines(mode, pl->n, lm, ln);
                const long wm = (lm + args.gtile - 1) / args.gtile, wn = (ln + args.gtile - 1) / args.gtile;
                sg.wg_begin = static_cast<int>(wg);
                sg.wg_main = static_cast<int>(wm);
                wg += (wm + wn) * sg.group;
            }
            if (wg > 0x7fffffffL) return PSPFFT_ERR_UNSUPPORTED_SIZE;
            args.nwg = static_cast<int>(wg);
            const size_t lds = bufs + (args.gtw ? ntw * csz : 0);
            PSPFFT_LOG(3, "pass %d prec %d generic: %d problems in %d segments, %ld workgroups of 256 threads, "
                          "%d lines each, %zu B LDS", mode, prec, args.count, args.nseg, wg, args.gtile, lds);
            // a whole number of rounds of 64 workgroups: the kernel deals its tiles to the XCDs in chunks
            const long grid = (wg + 63) / 64 * 64;
            if (grid > 0x7fffffffL) return PSPFFT_ERR_UNSUPPORTED_SIZE;
            if (pspfft::launch_generic(mode, prec, args, static_cast<int>(grid), lds, stream) != hipSuccess)
                return PSPFFT_ERR_DEVICE;
        }
    }
    return PSPFFT_OK;
}

// Grouped launches of a line pass (X_FWD .. X_INV kernels) for the problems idx.
pspfft_status launch_lines(int mode, const std::vector<int> &all_in, const pspfft_plan_t *plans,
                           const pspfft_workspace_t *ws, const void *const *S, void *const *Phi,
                           hipStream_t stream) {
    const int axis = pspfft::pass_axis(mode);
    const bool row = axis == 0;
    // axes outside the radix families go to the generic kernel
    std::vector<int> all, gen;
    for (int i : all_in) (plans[i]->host.ax[axis].E ? all : gen).push_back(i);
    if (!gen.empty()) {
        const pspfft_status st = launch_generic_lines(mode, gen, plans, ws, S, Phi, stream);
        if (st != PSPFFT_OK) return st;
    }
    // One kernel per (precision, radix family E, last-stage radix K, spectrum
    // layout); a kz-fastest z group also shares its lines' stage count (the
    // wavefront-owned kernel's tile depends on it).
    std::map<std::tuple<int, int, int, int>, std::vector<int>> groups;
    for (int i : all) {
        const AxisPlan &ax = plans[i]->host.ax[axis];
        const int K = ax.nst == 1 ? 1 : ax.R[ax.nst - 1];
        const int gz = mode == pspfft::Z_CONV && plans[i]->host.gz ? ax.nst : 0;
        groups[{static_cast<int>(plans[i]->prec), ax.E, K, gz}].push_back(i);
    }
    for (auto &kv : groups) {
        const int prec = std::get<0>(kv.first), E = std::get<1>(kv.first), K = std::get<2>(kv.first);
        const bool gz = std::get<3>(kv.first) != 0;
        std::vector<int> idx = kv.second;
        // problems of one plan next to each other: they form a segment sharing spectrum reads
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            return reinterpret_cast<uintptr_t>(plans[a]) < reinterpret_cast<uintptr_t>(plans[b]);
        });
        // Column passes: 128-byte rows of complex values per wavefront row.
        // Row passes: enough rows per workgroup for 256-thread groups.
        const int bmax = pspfft::max_block_for(prec, E);
        const int csz = prec == 0 ? 8 : 16;
        for (size_t c0 = 0; c0 < idx.size(); c0 += pspfft::kMaxProblems) {
            const size_t c1 = std::min(idx.size(), c0 + pspfft::kMaxProblems);
            int block = 0, nbmax = 1;
            for (size_t j = c0; j < c1; ++j) nbmax = std::max(nbmax, plans[idx[j]]->host.ax[axis].NB);
            // (a kz-fastest spectrum needs the compile-time tile: no override)
            const int gst = gz ? plans[idx[c0]]->host.ax[axis].nst : 0;
            const int tile_target = gz ? pspfft::wave_tile(prec, mode, E, nbmax, gst)
                                       : line_tile(mode, pspfft::pass_tile(prec, mode, E, nbmax));
            for (size_t j = c0; j < c1; ++j) block = std::max(block, tile_target * plans[idx[j]]->host.ax[axis].NB);
            block = std::min(std::max(block, 64), bmax);
            auto lds_need = [&](int blk) {
                size_t need = 0;
                for (size_t j = c0; j < c1; ++j) {
                    const AxisPlan &ax = plans[idx[j]]->host.ax[axis];
                    // wavefront-owned z lines: one row of wave_line_stride(L) per line
                    const size_t data = gz ? static_cast<size_t>(blk / ax.NB) * pspfft::wave_line_stride(ax.L)
                                           : static_cast<size_t>(pspfft::data_elems(row, ax.L, ax.NB, blk, csz));
                    const size_t e = data + ax.ntw + (row ? ax.L : 0);
                    need = std::max(need, e * csz);
                }
                return need;
            };
            while (block > nbmax && lds_need(block) > 160 * 1024) block /= 2;
            if (block < nbmax || lds_need(block) > 160 * 1024) return PSPFFT_ERR_UNSUPPORTED_SIZE;
            size_t lds = lds_need(block);
            LaunchArgs args;
            std::memset(&args, 0, sizeof(args));
            args.count = static_cast<int>(c1 - c0);
            args.nt = streaming_launch(plans, idx, c0, c1) ? 1 : 0;
            long wg = 0;
            for (size_t j = c0; j < c1; ++j) {
                const int i = idx[j];
                const pspfft_plan_t pl = plans[i];
                ProbArg &a = args.p[j - c0];
                a.plan = pl->dev;
                a.S = S ? S[i] : nullptr;
                a.Phi = Phi ? Phi[i] : nullptr;
                a.W = ws[i]->W;
                a.Wn = ws[i]->Wn;
                if (j > c0 && plans[idx[j - 1]] == pl) {
                    pspfft::Segment &sg = args.seg[args.nseg - 1];
                    sg.group += 1;
                    continue;
                }
                pspfft::Segment &sg = args.seg[args.nseg++];
                sg.first = static_cast<int>(j - c0);
                sg.group = 1;
            }
            for (int k = 0; k < args.nseg; ++k) {
                pspfft::Segment &sg = args.seg[k];
                const pspfft_plan_t pl = plans[idx[c0 + sg.first]];
                const int tile = block / pl->host.ax[axis].NB;
                long lm, ln;
                pass_lines(mode, pl->n, lm, ln);
                const long wm = (lm + tile - 1) / tile, wn = (ln + tile - 1) / tile;
                sg.wg_begin = static_cast<int>(wg);
                sg.wg_main = static_cast<int>(wm);
                wg += (wm + wn) * sg.group;
            }
            // grids are padded to a multiple of 8 (XCD renumbering) or 64 (chunked tile order)
            if (wg + 64 > 0x7fffffffL) return PSPFFT_ERR_UNSUPPORTED_SIZE;
            args.nwg = static_cast<int>(wg);
            args.xcd_remap = xcd_remap_mode(mode);
            args.wave_z = gz ? 1 : 0;
            const long align = args.xcd_remap == 1 ? 8 : (args.xcd_remap == 2 ? 64 : 1);
            const int grid = static_cast<int>((wg + align - 1) / align * align);
            // compile-time geometry when every line has two stages (radices E, K),
            // three (E, M, K) or four (E, M, M, K) and the workgroup holds
            // pass_tile() lines; 32-bit offsets when every array is below 4 GB
            // (else fix + kFixWide)
            const int M = E & -E;
            int fix = 0;
            if (K > 1) {
                const AxisPlan &a0 = plans[idx[c0]]->host.ax[axis];
                if (a0.nst == 2) fix = 2;
                else if (a0.nst == 3 && a0.R[1] == M) fix = 3;
                else if (a0.nst == 4 && a0.R[1] == M && a0.R[2] == M && M < E && E * M * M * K <= 4096) fix = 4;
                const int cnb = pspfft::fix_nb(fix, E, K);
                if (fix && !gz && block != pspfft::pass_tile(prec, mode, E, cnb) * cnb) fix = 0;
                if (fix && gz && block != pspfft::wave_tile(prec, mode, E, cnb, fix) * cnb) fix = 0;
                if (fix >= 3 && pspfft::pass_tile(prec, pspfft::Y_FWD, E, cnb) * cnb > pspfft::max_block_for(prec, E))
                    fix = 0;
                bool wide = false;
                for (size_t j = c0; j < c1 && fix; ++j) {
                    const AxisPlan &ax = plans[idx[j]]->host.ax[axis];
                    if (ax.nst != a0.nst || ax.NB != cnb) fix = 0;
                    if (!arrays_below_4gb(plans[idx[j]])) wide = true;
                }
                if (fix && wide) fix += pspfft::kFixWide;
            }
            // only wave_col_kernel reads that layout
            if (gz && (fix & 7) != 3 && (fix & 7) != 4) return PSPFFT_ERR_UNSUPPORTED_SIZE;
            // compile-time lines that keep their tables in global memory need only
            // their rows (or packed column positions) in LDS
            if (fix && row && pspfft::row_tables_global(prec, E, pspfft::fix_nb(fix, E, K))) {
                const AxisPlan &a0 = plans[idx[c0]]->host.ax[axis];
                lds = static_cast<size_t>(pspfft::data_elems(true, a0.L, a0.NB, block, csz)) * csz;
            }
            if (fix && !row && !gz && pspfft::col_tables_global(prec, mode, E, pspfft::fix_nb(fix, E, K))) {
                const AxisPlan &a0 = plans[idx[c0]]->host.ax[axis];
                lds = static_cast<size_t>(a0.L) * (block / a0.NB) * csz;
            }
            PSPFFT_LOG(3, "pass %d prec %d E %d K %d fix %d: %d problems in %d segments, %ld workgroups of %d "
                          "threads, %zu B LDS, streaming %d", mode, prec, E, K, fix, args.count, args.nseg, wg, block,
                       lds, args.nt);
            if (pspfft::launch_pass(mode, prec, E, K, fix, args, grid, block, lds, stream) != hipSuccess)
                return PSPFFT_ERR_DEVICE;
        }
    }
    return PSPFFT_OK;
}

// Grouped launches of the fused plane kernels (forward or inverse) for the problems idx.
pspfft_status launch_planes(bool fwd, const std::vector<int> &all, const pspfft_plan_t *plans,
                            const pspfft_workspace_t *ws, const void *const *S, void *const *Phi,
                            hipStream_t stream) {
    std::map<std::tuple<int, int, int>, std::vector<int>> groups;
    for (int i : all) groups[{static_cast<int>(plans[i]->prec), plans[i]->pE, plans[i]->pK}].push_back(i);
    for (auto &kv : groups) {
        const int prec = std::get<0>(kv.first), E = std::get<1>(kv.first), K = std::get<2>(kv.first);
        std::vector<int> idx = kv.second;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            return reinterpret_cast<uintptr_t>(plans[a]) < reinterpret_cast<uintptr_t>(plans[b]);
        });
        const size_t lds = pspfft::plane_lds_bytes(prec, E, K);
        for (size_t c0 = 0; c0 < idx.size(); c0 += pspfft::kMaxProblems) {
            const size_t c1 = std::min(idx.size(), c0 + pspfft::kMaxProblems);
            LaunchArgs args;
            std::memset(&args, 0, sizeof(args));
            args.count = static_cast<int>(c1 - c0);
            args.nt = streaming_launch(plans, idx, c0, c1) ? 1 : 0;
            for (size_t j = c0; j < c1; ++j) {
                const int i = idx[j];
                ProbArg &a = args.p[j - c0];
                a.plan = plans[i]->dev;
                a.S = S ? S[i] : nullptr;
                a.Phi = Phi ? Phi[i] : nullptr;
                a.W = ws[i]->W;
                a.Wn = ws[i]->Wn;
                if (j > c0 && plans[idx[j - 1]] == plans[i]) {
                    args.seg[args.nseg - 1].group += 1;
                    continue;
                }
                pspfft::Segment &sg = args.seg[args.nseg++];
                sg.first = static_cast<int>(j - c0);
                sg.group = 1;
            }
            long wg = 0;
            for (int k = 0; k < args.nseg; ++k) {  // one workgroup per z plane
                pspfft::Segment &sg = args.seg[k];
                const long nz = plans[idx[c0 + sg.first]]->n[2];
                sg.wg_begin = static_cast<int>(wg);
                sg.wg_main = static_cast<int>(nz);
                wg += nz * sg.group;
            }
            args.nwg = static_cast<int>(wg);
            PSPFFT_LOG(3, "plane %s prec %d E %d K %d: %d problems, %ld workgroups of %d threads, %zu B LDS, "
                          "streaming %d", fwd ? "fwd" : "inv", prec, E, K, args.count, wg, E * K * K, lds, args.nt);
            if (pspfft::launch_plane(fwd, prec, E, K, args, static_cast<int>(wg), lds, stream) != hipSuccess)
                return PSPFFT_ERR_DEVICE;
        }
    }
    return PSPFFT_OK;
}

// One pass for `count` problems.  Plans with fused planes run their x and y
// transforms together in X_FWD and X_INV and have nothing to do in Y_FWD and Y_INV.
pspfft_status run_pass(int mode, int count, const pspfft_plan_t *plans, const pspfft_workspace_t *ws,
                       const void *const *S, void *const *Phi, hipStream_t stream) {
    const pspfft_status bad = PSPFFT_ERR_INVALID_ARGUMENT;
    if (count < 0) return fail(bad, -1, "pass %d: negative count", mode);
    if (count == 0) return PSPFFT_OK;
    if (!plans || !ws) return fail(bad, -1, "pass %d: null plan or workspace array", mode);
    if (mode == pspfft::X_FWD && !S) return fail(bad, -1, "pass %d: null source array", mode);
    if (mode == pspfft::X_INV && !Phi) return fail(bad, -1, "pass %d: null potential array", mode);
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !ws[i] || ws[i]->plan != plans[i])
            return fail(bad, plans[i] ? plans[i]->verbosity : -1, "pass %d: problem %d: null plan or workspace, or a "
                        "workspace of another plan", mode, i);
        // the x passes move pairs of reals: S and Phi must be aligned to two reals
        const uintptr_t al = 2 * real_size(plans[i]->prec);
        if (mode == pspfft::X_FWD && (!S[i] || reinterpret_cast<uintptr_t>(S[i]) % al))
            return fail(bad, plans[i]->verbosity, "pass %d: problem %d: source null or not aligned to two reals", mode, i);
        if (mode == pspfft::X_INV && (!Phi[i] || reinterpret_cast<uintptr_t>(Phi[i]) % al))
            return fail(bad, plans[i]->verbosity, "pass %d: problem %d: potential null or not aligned to two reals", mode, i);
    }
    std::vector<int> lines, planes;
    for (int i = 0; i < count; ++i) {
        if (!plans[i]->fused || mode == pspfft::Z_CONV) lines.push_back(i);
        else if (mode == pspfft::X_FWD || mode == pspfft::X_INV) planes.push_back(i);
    }
    pspfft_status st = PSPFFT_OK;
    if (!planes.empty()) st = launch_planes(mode == pspfft::X_FWD, planes, plans, ws, S, Phi, stream);
    if (st == PSPFFT_OK && !lines.empty()) st = launch_lines(mode, lines, plans, ws, S, Phi, stream);
    if (st != PSPFFT_OK) return fail(st, plans[0]->verbosity, "pass %d of %d problems", mode, count);
    return PSPFFT_OK;
}


pspfft_status solve_all(int count, const pspfft_plan_t *plans, const pspfft_workspace_t *ws, const void *const *S,
                        void *const *Phi, hipStream_t stream);
pspfft_status check_batch(int count, const pspfft_plan_t *plans, const pspfft_workspace_t *ws, const void *const *S,
                          void *const *Phi);
pspfft_status solve_forked(const std::vector<std::vector<int>> &groups, const pspfft_plan_t *plans,
                           const pspfft_workspace_t *ws, const void *const *S, void *const *Phi, hipStream_t stream);

}  // namespace

extern "C" {

const char *pspfft_status_string(pspfft_status s) {
    switch (s) {
        case PSPFFT_OK: return "success";
        case PSPFFT_ERR_INVALID_ARGUMENT: return "invalid argument";
        case PSPFFT_ERR_UNSUPPORTED_SIZE: return "unsupported mesh size";
        case PSPFFT_ERR_OUT_OF_MEMORY: return "out of device memory";
        case PSPFFT_ERR_DEVICE: return "HIP device error";
        case PSPFFT_ERR_NOT_IMPLEMENTED: return "not implemented";
    }
    return "unknown status";
}

size_t pspfft_workspace_bytes(int nx, int ny, int nz, pspfft_precision prec) {
    if (prec != PSPFFT_FP32 && prec != PSPFFT_FP64) return 0;
    if (!sizes_ok(nx, ny, nz, prec)) return 0;
    const int n[3] = {nx, ny, nz};
    return ws_bytes(n, prec);
}

pspfft_status pspfft_plan_create(int nx, int ny, int nz, const double h[3], pspfft_precision prec,
                                 pspfft_plan_t *out) {
    return pspfft_plan_create_ex(nx, ny, nz, h, prec, PSPFFT_PLAN_DEFAULT, out);
}

pspfft_status pspfft_plan_create_ex(int nx, int ny, int nz, const double h[3], pspfft_precision prec,
                                    unsigned flags, pspfft_plan_t *out) {
    const unsigned vbits = (flags >> PSPFFT_PLAN_VERBOSITY_SHIFT) & 7u;
    const int vlevel = vbits ? static_cast<int>(vbits) - 1 : -1;
    const char *who = "pspfft_plan_create";
    if (!out || !h) return fail(PSPFFT_ERR_INVALID_ARGUMENT, vlevel, "%s: null %s", who, !out ? "out" : "h");
    if ((flags & ~(static_cast<unsigned>(PSPFFT_PLAN_FIVE_PASS) | (7u << PSPFFT_PLAN_VERBOSITY_SHIFT))) ||
        vbits > PSPFFT_CONSOLE_INFO_2 + 1)
        return fail(PSPFFT_ERR_INVALID_ARGUMENT, vlevel, "%s: unknown flags 0x%x", who, flags);
    if (prec != PSPFFT_FP32 && prec != PSPFFT_FP64)
        return fail(PSPFFT_ERR_INVALID_ARGUMENT, vlevel, "%s: unknown precision %d", who, static_cast<int>(prec));
    for (int a = 0; a < 3; ++a)
        if (!(std::isfinite(h[a]) && h[a] > 0.0))
            return fail(PSPFFT_ERR_INVALID_ARGUMENT, vlevel, "%s: cell width h[%d] = %g is not finite and positive",
                        who, a, h[a]);
    if (nx < 1 || ny < 1 || nz < 1)
        return fail(PSPFFT_ERR_INVALID_ARGUMENT, vlevel, "%s: mesh %d x %d x %d", who, nx, ny, nz);
    if (!sizes_ok(nx, ny, nz, prec))
        return fail(PSPFFT_ERR_UNSUPPORTED_SIZE, vlevel,
                    "%s: mesh %d x %d x %d (each size must be 2^a 3^b 5^c, at most 2048; rows of up to %d with odd "
                    "part 1, 3, 5 or 9)", who, nx, ny, nz, 2 * max_n(prec));

    pspfft_plan_t p = new (std::nothrow) pspfft_plan_s();
    if (!p) return fail(PSPFFT_ERR_OUT_OF_MEMORY, vlevel, "%s: host allocation", who);
    auto guard = make_guard([&] { destroy_plan(p); });
    p->verbosity = vlevel;
    p->n[0] = nx;
    p->n[1] = ny;
    p->n[2] = nz;
    for (int a = 0; a < 3; ++a) p->h[a] = h[a];
    p->prec = prec;
    const size_t rs = real_size(prec), cs = cplx_size(prec);
    std::memset(&p->host, 0, sizeof(p->host));
    p->host.nx = nx;
    p->host.ny = ny;
    p->host.nz = nz;
    p->host.prec = prec == PSPFFT_FP32 ? 0 : 1;
    size_t bytes = 0;
    const char *pname = prec == PSPFFT_FP32 ? "fp32" : "fp64";
    PSPFFT_MSG(vlevel, PSPFFT_CONSOLE_INFO_1, "creating plan %d x %d x %d %s, h = (%g, %g, %g)", nx, ny, nz, pname,
               h[0], h[1], h[2]);

    // stage plans and twiddle tables (FP64, rounded once to the plan precision)
    std::vector<std::complex<double>> tws[3];
    for (int a = 0; a < 3; ++a) {
        if (!build_axis(a, p->n[a], prec, p->host.ax[a], tws[a]))
            return fail(PSPFFT_ERR_UNSUPPORTED_SIZE, vlevel, "%s: no stage plan for axis %d (n = %d)", who, a,
                        p->n[a]);
        if (a == 2 && z32_enabled() && prec == PSPFFT_FP32 && p->host.ax[2].E == 16 && p->host.ax[2].L == 2048) {
            // the 32-family's z lines, where the wavefront-owned z kernel takes them
            const AxisPlan keep = p->host.ax[2];
            std::vector<std::complex<double>> tw32;
            if (build_axis(2, p->n[2], prec, p->host.ax[2], tw32, 32) && z_wave_lines(p))
                tws[2].swap(tw32);
            else
                p->host.ax[2] = keep;
        }
        const AxisPlan &ax = p->host.ax[a];
        char radices[96] = {0};
        for (int s2 = 0, off = 0; s2 < ax.nst && off < 90; ++s2)
            off += std::snprintf(radices + off, sizeof(radices) - off, s2 ? " x %d" : "%d", ax.R[s2]);
        PSPFFT_MSG(vlevel, PSPFFT_CONSOLE_INFO_2, "  axis %c: n = %d, line of %d points, stages %s, %s", "xyz"[a],
                   ax.n, ax.L, ax.nst ? radices : "none", ax.E ? "radix-family kernels" : "generic line kernel");
        if (!ax.E)
            PSPFFT_MSG(vlevel, PSPFFT_CONSOLE_WARNING,
                       "plan %d x %d x %d %s: axis %c (n = %d) runs on the generic line kernel, slower than the "
                       "radix families (n = 2^a times 1, 3, 5 or 9)", nx, ny, nz, pname, "xyz"[a], ax.n);
    }
    if (hipGetDevice(&p->device) != hipSuccess) return fail(PSPFFT_ERR_DEVICE, vlevel, "%s: hipGetDevice", who);
    for (int a = 0; a < 3; ++a) {
        const std::vector<std::complex<double>> &tw = tws[a];
        const size_t tb = tw.size() * cs;
        pspfft_status st = alloc(&p->tw[a], tb);
        if (st != PSPFFT_OK) return fail(st, vlevel, "%s: twiddle table of %zu bytes", who, tb);
        std::vector<unsigned char> buf(tb);
        for (size_t i = 0; i < tw.size(); ++i) {
            if (prec == PSPFFT_FP32) {
                const float v[2] = {static_cast<float>(tw[i].real()), static_cast<float>(tw[i].imag())};
                std::memcpy(&buf[i * cs], v, sizeof(v));
            } else {
                const double v[2] = {tw[i].real(), tw[i].imag()};
                std::memcpy(&buf[i * cs], v, sizeof(v));
            }
        }
        if (hipMemcpy(p->tw[a], buf.data(), tb, hipMemcpyHostToDevice) != hipSuccess)
            return fail(PSPFFT_ERR_DEVICE, vlevel, "%s: twiddle upload", who);
        p->host.ax[a].tw = p->tw[a];
        p->host.ax[a].post = a == 0 ? static_cast<char *>(p->tw[a]) + p->host.ax[a].ntw * cs : nullptr;
        bytes += tb;
    }
    // Workspace z tiles.  Only meshes whose z planes span 4 MB or more are
    // tiled: there the z lines of the z pass miss the address translation
    // caches, while for smaller planes the wider row stride costs more than it
    // saves.  The tile is the largest power of two up to 16 (PSPFFT_ZTILE
    // overrides the cap) dividing the z lines' threads per line.
    {
        const size_t plane = static_cast<size_t>(2) * ny * nx * cs;
        int cap = plane >= (size_t(4) << 20) ? 16 : 1;
        if (const char *e = std::getenv("PSPFFT_ZTILE")) {
            const int v = std::atoi(e);
            if (v >= 1 && v <= 16 && (v & (v - 1)) == 0) cap = v;
        }
        const int nbz = p->host.ax[2].NB;
        int zb = 1;  // generic z lines (NB = 0): no tiling, nz need not be a multiple of anything
        while (nbz > 0 && zb < cap && nbz % (2 * zb) == 0) zb *= 2;
        p->host.zb = zb;
    }
    // kz-fastest spectrum for wavefront-owned z lines and for z lines on the
    // generic kernel (whose lanes of a line walk consecutive kz)
    p->host.gz = z_wave_lines(p) || p->host.ax[2].E == 0 ? 1 : 0;
    // fused x-y plane kernels: nx == ny = E*K (at most two stages) and the plane fits in LDS
    {
        const AxisPlan &ax = p->host.ax[0];
        const int K = ax.nst == 1 ? 1 : ax.R[1];
        p->fused = !(flags & PSPFFT_PLAN_FIVE_PASS) && nx == ny && ax.nst <= 2 && ax.E * K == nx &&
                   ax.ntw == nx - 1 && pspfft::plane_fits(p->host.prec, ax.E, K) && p->host.zb == 1;
        if (p->fused) {
            p->pE = ax.E;
            p->pK = K;
        }
    }

    // Green's-function spectrum, computed once in FP64 and kept (Sec. 2.2.2)
    const size_t oct = static_cast<size_t>(nx + 1) * (ny + 1) * (nz + 1);
    const size_t gmain = static_cast<size_t>(nz + 1) * (ny + 1) * nx * rs;
    const size_t gnyq = static_cast<size_t>(nz + 1) * (ny + 1) * rs;
    pspfft_status st;
    if ((st = alloc(&p->G, gmain)) != PSPFFT_OK || (st = alloc(&p->Gn, gnyq)) != PSPFFT_OK)
        return fail(st, vlevel, "%s: spectrum of %zu bytes", who, gmain + gnyq);
    bytes += gmain + gnyq;
    {
        void *a = nullptr, *b = nullptr, *cx = nullptr, *cy = nullptr, *cz = nullptr;
        hipStream_t s = nullptr;
        auto tmp = make_guard([&] {
            if (s) (void)hipStreamDestroy(s);
            for (void *q : {a, b, cx, cy, cz})
                if (q) (void)hipFree(q);
        });
        const std::vector<double> tx = cos_table(nx), ty = cos_table(ny), tz = cos_table(nz);
        if ((st = alloc(&a, oct * sizeof(double))) != PSPFFT_OK || (st = alloc(&b, oct * sizeof(double))) != PSPFFT_OK ||
            (st = alloc(&cx, tx.size() * sizeof(double))) != PSPFFT_OK ||
            (st = alloc(&cy, ty.size() * sizeof(double))) != PSPFFT_OK ||
            (st = alloc(&cz, tz.size() * sizeof(double))) != PSPFFT_OK)
            return fail(st, vlevel, "%s: FP64 spectrum scratch of %zu bytes", who, 2 * oct * sizeof(double));
        if (hipMemcpy(cx, tx.data(), tx.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(cy, ty.data(), ty.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(cz, tz.data(), tz.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
            pspfft::green_spectrum(nx, ny, nz, p->h, p->host.prec, p->host.gz, static_cast<double *>(a),
                                   static_cast<double *>(b), static_cast<const double *>(cx),
                                   static_cast<const double *>(cy), static_cast<const double *>(cz), p->G, p->Gn,
                                   s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(PSPFFT_ERR_DEVICE, vlevel, "%s: spectrum of the doubled Green's function", who);
    }
    p->host.G = p->G;
    p->host.Gn = p->Gn;

    void *dv = nullptr;
    if ((st = alloc(&dv, sizeof(DevPlan))) != PSPFFT_OK) return fail(st, vlevel, "%s: plan table", who);
    p->dev = static_cast<DevPlan *>(dv);
    if (hipMemcpy(p->dev, &p->host, sizeof(DevPlan), hipMemcpyHostToDevice) != hipSuccess)
        return fail(PSPFFT_ERR_DEVICE, vlevel, "%s: plan table upload", who);
    bytes += sizeof(DevPlan);
    p->bytes = bytes;  // the default workspace comes with the first pspfft_solve

    PSPFFT_MSG(vlevel, PSPFFT_CONSOLE_INFO_1,
               "plan %d x %d x %d %s: %zu bytes resident, %s, spectrum %s, workspace %zu bytes per solve "
               "(z tile %d)", nx, ny, nz, pname, bytes, p->fused ? "fused x-y planes" : "five passes",
               p->host.gz ? "kz-fastest" : "kx-fastest", ws_bytes(p->n, prec), p->host.zb);
    guard.armed = false;
    *out = p;
    return PSPFFT_OK;
}

pspfft_status pspfft_destroy(pspfft_plan_t plan) {
    if (!plan) return fail(PSPFFT_ERR_INVALID_ARGUMENT, -1, "pspfft_destroy: null plan");
    PSPFFT_MSG(plan->verbosity, PSPFFT_CONSOLE_INFO_1, "destroying plan %d x %d x %d %s", plan->n[0], plan->n[1],
               plan->n[2], plan->prec == PSPFFT_FP32 ? "fp32" : "fp64");
    destroy_plan(plan);
    return PSPFFT_OK;
}

pspfft_status pspfft_workspace_create(pspfft_plan_t plan, pspfft_workspace_t *out) {
    if (!plan || !out) return fail(PSPFFT_ERR_INVALID_ARGUMENT, plan ? plan->verbosity : -1, "pspfft_workspace_create: null argument");
    pspfft_workspace_t w = new (std::nothrow) pspfft_workspace_s();
    if (!w) return fail(PSPFFT_ERR_OUT_OF_MEMORY, plan->verbosity, "pspfft_workspace_create: host allocation");
    w->plan = plan;
    w->owned = true;
    w->bytes = ws_bytes(plan->n, plan->prec);
    pspfft_status st = alloc(&w->mem, w->bytes);
    if (st != PSPFFT_OK) {
        delete w;
        return fail(st, plan->verbosity, "pspfft_workspace_create: %zu bytes", ws_bytes(plan->n, plan->prec));
    }
    ws_split(w, plan->n, plan->prec);
    *out = w;
    return PSPFFT_OK;
}

pspfft_status pspfft_workspace_wrap(pspfft_plan_t plan, void *memory, size_t bytes, pspfft_workspace_t *out) {
    if (!plan || !memory || !out) return fail(PSPFFT_ERR_INVALID_ARGUMENT, plan ? plan->verbosity : -1, "pspfft_workspace_wrap: null argument");
    if (bytes < ws_bytes(plan->n, plan->prec))
        return fail(PSPFFT_ERR_INVALID_ARGUMENT, plan->verbosity, "pspfft_workspace_wrap: %zu bytes, the plan needs %zu",
                    bytes, ws_bytes(plan->n, plan->prec));
    if (reinterpret_cast<uintptr_t>(memory) % 256 != 0)
        return fail(PSPFFT_ERR_INVALID_ARGUMENT, plan->verbosity, "pspfft_workspace_wrap: memory not 256-byte aligned");
    pspfft_workspace_t w = new (std::nothrow) pspfft_workspace_s();
    if (!w) return fail(PSPFFT_ERR_OUT_OF_MEMORY, plan->verbosity, "pspfft_workspace_wrap: host allocation");
    w->plan = plan;
    w->owned = false;
    w->mem = memory;
    w->bytes = bytes;
    ws_split(w, plan->n, plan->prec);
    *out = w;
    return PSPFFT_OK;
}

pspfft_status pspfft_workspace_destroy(pspfft_workspace_t ws) {
    if (!ws) return fail(PSPFFT_ERR_INVALID_ARGUMENT, -1, "pspfft_workspace_destroy: null workspace");
    if (ws->plan && ws == ws->plan->ws)
        return fail(PSPFFT_ERR_INVALID_ARGUMENT, ws->plan->verbosity,
                    "pspfft_workspace_destroy: the plan's default workspace goes with the plan");
    if (ws->owned && ws->mem) (void)hipFree(ws->mem);  // after the work queued on the device
    delete ws;
    return PSPFFT_OK;
}

pspfft_status pspfft_pass_batched(pspfft_pass pass, int count, const pspfft_plan_t *plans,
                                  const pspfft_workspace_t *ws, const void *const *S, void *const *Phi,
                                  hipStream_t stream) {
    if (pass < PSPFFT_PASS_X_FWD || pass > PSPFFT_PASS_X_INV)
        return fail(PSPFFT_ERR_INVALID_ARGUMENT, -1, "pspfft_pass_batched: unknown pass %d", static_cast<int>(pass));
    return run_pass(static_cast<int>(pass), count, plans, ws, S, Phi, stream);
}

pspfft_status pspfft_solve_batched(int count, const pspfft_plan_t *plans, const pspfft_workspace_t *ws,
                                   const void *const *S, void *const *Phi, hipStream_t stream) {
    pspfft_status st = check_batch(count, plans, ws, S, Phi);
    if (st != PSPFFT_OK) return st;
    // problems of one plan form a group; several groups run side by side
    std::vector<pspfft_plan_t> keys;
    std::vector<std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
        size_t g = 0;
        while (g < keys.size() && keys[g] != plans[i]) ++g;
        if (g == keys.size()) {
            keys.push_back(plans[i]);
            groups.emplace_back();
        }
        groups[g].push_back(i);
    }
    if (groups.size() < 2) return solve_all(count, plans, ws, S, Phi, stream);
    return solve_forked(groups, plans, ws, S, Phi, stream);
}

}  // extern "C"

namespace {
// Every argument of a batch of whole solves, checked before anything is
// enqueued: plans and their own distinct workspaces, sources and potentials
// present and aligned to two reals.
pspfft_status check_batch(int count, const pspfft_plan_t *plans, const pspfft_workspace_t *ws, const void *const *S,
                          void *const *Phi) {
    const pspfft_status bad = PSPFFT_ERR_INVALID_ARGUMENT;
    if (count < 0 || (count > 0 && (!plans || !ws || !S || !Phi)))
        return fail(bad, -1, "pspfft_solve_batched: count %d or null array", count);
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !ws[i] || ws[i]->plan != plans[i])
            return fail(bad, plans[i] ? plans[i]->verbosity : -1, "pspfft_solve_batched: problem %d: null plan or "
                        "workspace, or a workspace of another plan", i);
        const uintptr_t al = 2 * real_size(plans[i]->prec);
        if (!S[i] || !Phi[i] || reinterpret_cast<uintptr_t>(S[i]) % al || reinterpret_cast<uintptr_t>(Phi[i]) % al)
            return fail(bad, plans[i]->verbosity, "pspfft_solve_batched: problem %d: source or potential null or not "
                        "aligned to two reals", i);
        for (int j = i + 1; j < count; ++j)
            if (ws[i] == ws[j])
                return fail(bad, -1, "pspfft_solve_batched: problems %d and %d share a workspace", i, j);
    }
    return PSPFFT_OK;
}

pspfft_status solve_all(int count, const pspfft_plan_t *plans, const pspfft_workspace_t *ws, const void *const *S,
                        void *const *Phi, hipStream_t stream) {
    pspfft_status st = check_batch(count, plans, ws, S, Phi);
    for (int mode = pspfft::X_FWD; st == PSPFFT_OK && mode <= pspfft::X_INV; ++mode)
        st = run_pass(mode, count, plans, ws, S, Phi, stream);
    return st;
}

// Streams and events for batches that run several plans side by side: per
// device, kForkStreams non-blocking streams of default priority and a ring of
// events, created on first use.  A fork records an event on the caller's
// stream that every group's stream waits for, enqueues each group's five
// passes on its stream, and makes the caller's stream wait for each stream's
// last event, so the batch is ordered after the caller's earlier work and
// before its later work, as on one stream.  (A wait takes the event as recorded
// at the time of the call, so reusing the ring's events later is safe.)
constexpr int kForkStreams = 8;
constexpr int kForkEvents = 64;
struct ForkPool {
    std::mutex mu;
    hipStream_t streams[kForkStreams] = {};
    hipEvent_t events[kForkEvents] = {};
    int next = 0;
    bool ready = false;
};
ForkPool g_fork[64];

pspfft_status solve_forked(const std::vector<std::vector<int>> &groups, const pspfft_plan_t *plans,
                           const pspfft_workspace_t *ws, const void *const *S, void *const *Phi, hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(PSPFFT_ERR_DEVICE, -1, "pspfft_solve_batched: hipGetDevice");
    ForkPool &fp = g_fork[dev];
    std::lock_guard<std::mutex> lk(fp.mu);
    if (!fp.ready) {
        for (auto &q : fp.streams)
            if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess)
                return fail(PSPFFT_ERR_DEVICE, -1, "pspfft_solve_batched: stream creation");
        for (auto &e : fp.events)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return fail(PSPFFT_ERR_DEVICE, -1, "pspfft_solve_batched: event creation");
        fp.ready = true;
    }
    auto event = [&]() {
        hipEvent_t e = fp.events[fp.next];
        fp.next = (fp.next + 1) % kForkEvents;
        return e;
    };
    const hipEvent_t start = event();
    if (hipEventRecord(start, stream) != hipSuccess) return fail(PSPFFT_ERR_DEVICE, -1, "pspfft_solve_batched: fork");
    const int nused = static_cast<int>(std::min<size_t>(groups.size(), kForkStreams));
    for (int k = 0; k < nused; ++k)
        if (hipStreamWaitEvent(fp.streams[k], start, 0) != hipSuccess)
            return fail(PSPFFT_ERR_DEVICE, -1, "pspfft_solve_batched: fork");
    pspfft_status st = PSPFFT_OK;
    for (size_t g = 0; g < groups.size() && st == PSPFFT_OK; ++g) {
        std::vector<pspfft_plan_t> p;
        std::vector<pspfft_workspace_t> w;
        std::vector<const void *> s;
        std::vector<void *> f;
        for (int i : groups[g]) {
            p.push_back(plans[i]);
            w.push_back(ws[i]);
            s.push_back(S[i]);
            f.push_back(Phi[i]);
        }
        st = solve_all(static_cast<int>(p.size()), p.data(), w.data(), s.data(), f.data(),
                       fp.streams[g % kForkStreams]);
    }
    // join every stream that took work, whatever happened above
    for (int k = 0; k < nused; ++k) {
        const hipEvent_t done = event();
        if (hipEventRecord(done, fp.streams[k]) != hipSuccess || hipStreamWaitEvent(stream, done, 0) != hipSuccess)
            st = fail(PSPFFT_ERR_DEVICE, -1, "pspfft_solve_batched: join");
    }
    return st;
}
}  // namespace

extern "C" {

pspfft_status pspfft_solve_ws(pspfft_plan_t plan, pspfft_workspace_t ws, const void *S, void *Phi,
                              hipStream_t stream) {
    if (!plan || !ws || !S || !Phi) return fail(PSPFFT_ERR_INVALID_ARGUMENT, plan ? plan->verbosity : -1, "pspfft_solve_ws: null argument");
    return pspfft_solve_batched(1, &plan, &ws, &S, &Phi, stream);
}

pspfft_status pspfft_solve(pspfft_plan_t plan, const void *S, void *Phi, hipStream_t stream) {
    if (!plan || !S || !Phi) return fail(PSPFFT_ERR_INVALID_ARGUMENT, plan ? plan->verbosity : -1, "pspfft_solve: null argument");
    pspfft_workspace_t ws;
    {
        std::lock_guard<std::mutex> lk(plan->mu);
        if (!plan->ws) {  // the default workspace, on first use
            pspfft_workspace_t w = new (std::nothrow) pspfft_workspace_s();
            if (!w) return fail(PSPFFT_ERR_OUT_OF_MEMORY, plan->verbosity, "pspfft_solve: host allocation");
            w->plan = plan;
            w->owned = true;
            w->bytes = ws_bytes(plan->n, plan->prec);
            const pspfft_status st = alloc(&w->mem, w->bytes);
            if (st != PSPFFT_OK) {
                delete w;
                return fail(st, plan->verbosity, "pspfft_solve: default workspace of %zu bytes", ws_bytes(plan->n, plan->prec));
            }
            ws_split(w, plan->n, plan->prec);
            plan->ws = w;
        }
        ws = plan->ws;
    }
    return pspfft_solve_ws(plan, ws, S, Phi, stream);
}

size_t pspfft_plan_resident_bytes(int nx, int ny, int nz, pspfft_precision prec) {
    if (prec != PSPFFT_FP32 && prec != PSPFFT_FP64) return 0;
    if (!sizes_ok(nx, ny, nz, prec)) return 0;
    const int n[3] = {nx, ny, nz};
    size_t bytes = sizeof(DevPlan);
    for (int a = 0; a < 3; ++a) {  // twiddle tables, as pspfft_plan_create builds them
        AxisPlan ax;
        std::vector<std::complex<double>> tw;
        if (!build_axis(a, n[a], prec, ax, tw)) return 0;
        bytes += tw.size() * cplx_size(prec);
    }
    // spectrum octant: main part and the kx = nx column
    bytes += static_cast<size_t>(nz + 1) * (ny + 1) * (nx + 1) * real_size(prec);
    return bytes;
}

size_t pspfft_plan_bytes(pspfft_plan_t plan) {
    if (!plan) return 0;
    std::lock_guard<std::mutex> lk(plan->mu);
    return plan->bytes + (plan->ws ? plan->ws->bytes : 0);
}

size_t pspfft_pass_bytes(pspfft_plan_t plan, pspfft_pass pass) {
    if (!plan) return 0;
    const size_t r = real_size(plan->prec), c = cplx_size(plan->prec);
    const size_t nx = plan->n[0], ny = plan->n[1], nz = plan->n[2];
    const size_t half = ny * nz * (nx + 1) * c;  // spectrum rows y < ny (kx <= nx)
    const size_t full = 2 * half;                // all 2ny rows
    if (plan->fused) {  // x and y transforms of a plane in one pass; no intermediate in HBM
        switch (pass) {
            case PSPFFT_PASS_X_FWD: return nx * ny * nz * r + full;
            case PSPFFT_PASS_Z_CONV: return 2 * full + (nx + 1) * (ny + 1) * (nz + 1) * r;
            case PSPFFT_PASS_X_INV: return full + nx * ny * nz * r;
            default: return 0;
        }
    }
    switch (pass) {
        case PSPFFT_PASS_X_FWD: return nx * ny * nz * r + half;
        case PSPFFT_PASS_Y_FWD: return half + full;
        case PSPFFT_PASS_Z_CONV: return 2 * full + (nx + 1) * (ny + 1) * (nz + 1) * r;
        case PSPFFT_PASS_Y_INV: return full + half;
        case PSPFFT_PASS_X_INV: return half + nx * ny * nz * r;
    }
    return 0;
}

int pspfft_plan_fused(pspfft_plan_t plan) { return plan && plan->fused ? 1 : 0; }

int pspfft_plan_spectrum_kz_fastest(pspfft_plan_t plan) { return plan && plan->host.gz ? 1 : 0; }

int pspfft_workspace_ztile(pspfft_plan_t plan) { return plan ? plan->host.zb : 0; }

pspfft_status pspfft_plan_info(pspfft_plan_t plan, int dims[3], double h[3], pspfft_precision *prec) {
    if (!plan) return PSPFFT_ERR_INVALID_ARGUMENT;
    for (int a = 0; a < 3; ++a) {
        if (dims) dims[a] = plan->n[a];
        if (h) h[a] = plan->h[a];
    }
    if (prec) *prec = plan->prec;
    return PSPFFT_OK;
}

pspfft_status pspfft_set_verbosity(pspfft_verbosity level) {
    if (level < PSPFFT_CONSOLE_ERROR || level > PSPFFT_CONSOLE_INFO_2)
        return fail(PSPFFT_ERR_INVALID_ARGUMENT, -1, "pspfft_set_verbosity: unknown level %d", static_cast<int>(level));
    g_level.store(static_cast<int>(level), std::memory_order_relaxed);
    return PSPFFT_OK;
}

pspfft_verbosity pspfft_get_verbosity(void) { return static_cast<pspfft_verbosity>(process_level()); }

pspfft_status pspfft_set_log_callback(pspfft_log_fn fn, void *user) {
    std::lock_guard<std::mutex> lk(g_log_mu);
    g_log_fn = fn;
    g_log_user = fn ? user : nullptr;
    return PSPFFT_OK;
}

pspfft_status pspfft_plan_green(pspfft_plan_t plan, void *dst, hipStream_t stream) {
    if (!plan || !dst) return PSPFFT_ERR_INVALID_ARGUMENT;
    if (pspfft::green_export(plan->n[0], plan->n[1], plan->n[2], plan->host.prec, plan->host.gz, plan->G, plan->Gn,
                             dst, stream) != hipSuccess)
        return PSPFFT_ERR_DEVICE;
    return PSPFFT_OK;
}

}  // extern "C"

namespace pspfft {
// Report a failure about `plan` at level error (for entry points defined in
// other files) and return its status.
pspfft_status report_failure(pspfft_status st, pspfft_plan_t plan, const char *what) {
    return fail(st, plan ? plan->verbosity : -1, "%s", what);
}

// One solve with `bytes` bytes of device memory at `mem` (256-byte aligned) as
// its workspace, through a workspace handle on the stack: allocates nothing.
pspfft_status solve_on(pspfft_plan_t plan, void *mem, size_t bytes, const void *S, void *Phi, hipStream_t stream) {
    if (!plan || !mem || !S || !Phi) return fail(PSPFFT_ERR_INVALID_ARGUMENT, plan ? plan->verbosity : -1, "solve: null argument");
    if (bytes < ws_bytes(plan->n, plan->prec) || reinterpret_cast<uintptr_t>(mem) % 256 != 0)
        return fail(PSPFFT_ERR_INVALID_ARGUMENT, plan->verbosity, "solve: workspace memory too small or misaligned");
    pspfft_workspace_s w;  // a handle on the stack: no allocation
    w.plan = plan;
    w.owned = false;
    w.mem = mem;
    w.bytes = bytes;
    ws_split(&w, plan->n, plan->prec);
    pspfft_workspace_t wp = &w;
    return solve_all(1, &plan, &wp, &S, &Phi, stream);
}
}  // namespace pspfft
