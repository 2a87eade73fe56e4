// plane_kernels.h -- the x and y transforms of one z plane in one workgroup,
// for meshes with nx == ny = n whose plane of x spectra fits in LDS (Sec. 2.1
// and 2.2.2: the same transforms as the x and y passes, without the round trip
// of the intermediate through HBM).
//
// Forward (source plane -> W rows ky < 2n):
//   x step : the n rows are transformed as in the x pass (packed real form and
//            split step); X[y][kx], kx < n, lands in the LDS plane, and the real
//            values X[y][0] and X[y][n] share the slot of kx = 0 as X0 + i Xn.
//   y step : a zero-padded length-2n transform equals two length-n transforms:
//            Y[2j] = DFT_n(x)[j] and Y[2j+1] = DFT_n(x[y] e^{-i pi y/n})[j].
//            Each runs with its exchange inside the column's own n LDS slots,
//            so the plane needs no extra room.  Column 0 carries the transform
//            C of X0 + i Xn; its threads, lanes of one wavefront, separate the two
//            real columns as they store them, with A[k] = (C[k] + conj C[-k])/2
//            and B[k] = (C[k] - conj C[-k])/(2i), the partners C[-k] coming from
//            other lanes.
// Inverse (W rows -> potential plane):
//   y step : x[y] = IDFT_n(Y[2j])[y] + e^{+i pi y/n} IDFT_n(Y[2j+1])[y], y < n.
//            Columns kx = 0 and kx = n have real results, so they are
//            transformed together as Y0 + i Yn and come out as x0 + i xn.
//   x step : the inverse split step and the inverse x transform of each row,
//            x < n kept.
//
// n = E*K: at most two stages, NB = K threads per line, n*K threads per
// workgroup; the geometry is compile-time.
#pragma once

#include <cstdlib>

#include "pass_kernels.h"

namespace pspfft {

// Keep a lane offset opaque to loop-invariant code motion, so that the
// per-element offsets derived from it are recomputed inside the plane loop
// (one add each) instead of being hoisted out and held in registers.
template <typename I>
__device__ __forceinline__ void opaque(I &v) { asm volatile("" : "+v"(v)); }

// Element at byte offset `off` (32 bits) from a base pointer that is the same
// for the whole workgroup, so the address is a scalar base plus one 32-bit
// vector offset instead of a 64-bit vector address per element.
template <typename T>
__device__ __forceinline__ const cx<T> &at(const void *base, uint32_t off) {
    return *reinterpret_cast<const cx<T> *>(static_cast<const char *>(base) + off);
}
template <typename T>
__device__ __forceinline__ cx<T> &at(void *base, uint32_t off) {
    return *reinterpret_cast<cx<T> *>(static_cast<char *>(base) + off);
}

// Problem and z of plane `pl` of a launch (segments are numbered plane-major
// within a run of problems that share a plan).
struct PlaneRef {
    const ProbArg *pa;
    int z;
};
__device__ __forceinline__ PlaneRef plane_ref(const LaunchArgs &args, int pl) {
    int sgi = 0;
    while (sgi + 1 < args.nseg && pl >= args.seg[sgi + 1].wg_begin) ++sgi;
    const Segment &sg = args.seg[sgi];
    const int local = pl - sg.wg_begin;
    return PlaneRef{&args.p[sg.first + local % sg.group], local / sg.group};
}

// Each workgroup takes planes blockIdx.x, blockIdx.x + gridDim.x, ...  The
// forward kernel loads the next source plane before it stores the current one,
// so the loads complete under the y transforms (the compiler's wait for them
// still covers most of the stores issued after them).  The inverse kernel loads the odd W rows of a plane while it transforms the even
// ones, and the next plane's even rows (and Nyquist column) during the x step;
// a whole plane of input would not fit in registers beside the one in use.
// NT (inverse planes of a streaming launch): the W rows are loaded with
// nontemporal accesses; they are read once.
template <typename T, int E, int K, bool FWD, bool NT = false>
__global__ void __launch_bounds__(E * K * K) plane_kernel(const LaunchArgs args) {
    constexpr int n = E * K;
    constexpr int NB = K;
    constexpr int H = E / 2;
    constexpr int BLK = E * K * K;  // threads: n lines of NB threads
    constexpr int CSZ = static_cast<int>(sizeof(cx<T>));
    constexpr int SP = row_stride(n, NB, CSZ);  // LDS row stride of the plane
    using RowF = LineFFT<T, E, -1, true, NB, SP>;
    using RowI = LineFFT<T, E, +1, true, NB, SP>;
    using ColF = LineFFT<T, E, -1, false, NB, SP>;
    using ColI = LineFFT<T, E, +1, false, NB, SP>;

    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem);

    const int G = static_cast<int>(gridDim.x);
    int pl = static_cast<int>(blockIdx.x);
    if (pl >= args.nwg) return;

    // stage twiddles (n - 1 entries), exp(-i pi k / n) (k < n), and 2n slots for
    // the Nyquist column (inverse).  The tables depend on n only, so every
    // problem of the launch shares them.
    const AxisPlan &ax = args.p[0].plan->ax[0];
    cx<T> *twl = lds + n * SP;
    const cx<T> *post = twl + (n - 1);
    copy_to_lds<T>(twl, ax.tw, 2 * n - 1);

    int tid = static_cast<int>(threadIdx.x);
    // x step: row y = xc, thread xt of the row; y step: column kx = yc, thread yt
    // of the column, at position cp within an LDS row.  Recomputed per plane
    // from an opaque tid (see opaque()).
    int xc, xt, yc, yt, cp;
    auto lanes = [&]() {
        opaque(tid);
        xc = tid / NB;
        xt = tid % NB;
        yc = tid % n;
        yt = tid / n;
        if constexpr (FWD) {
            // the NB threads of column 0 are lanes 0..NB-1 of wavefront 0 (threads
            // 1..NB-1 trade places with the first threads of columns 1..NB-1)
            if (yt == 0 && yc >= 1 && yc < NB) {
                yt = yc;
                yc = 0;
            } else if (yc == 0 && yt >= 1) {
                yc = yt;
                yt = 0;
            }
        }
        cp = yc + (yc >> 4);
    };
    lanes();

    // z plane of the workspace: fused plans have untiled workspaces (one z plane
    // per tile), so rows ky are n values apart
    auto W_of = [&](const PlaneRef &r) { return static_cast<cx<T> *>(r.pa->W) + static_cast<size_t>(r.z) * 2 * n * n; };
    auto rs_of = [&](const PlaneRef &) { return static_cast<uint32_t>(n * CSZ); };
    auto Wn_of = [&](const PlaneRef &r) { return static_cast<cx<T> *>(r.pa->Wn) + static_cast<size_t>(r.z) * 2 * n; };

    if constexpr (FWD) {
        cx<T> s[H];  // this thread's packed source values of the current plane
        auto load_src = [&](int p) {
            const PlaneRef r = plane_ref(args, p);
            const uint32_t src_off = static_cast<uint32_t>((xc * n + 2 * xt) * sizeof(T));
            const void *plane = static_cast<const T *>(r.pa->S) + static_cast<size_t>(r.z) * n * n;
#pragma unroll
            for (int m = 0; m < H; ++m) s[m] = at<T>(plane, src_off + m * NB * CSZ);
        };
        // FP32: the next plane's source is loaded during the y step (below); FP64
        // loads it here, where the 16-byte values need no registers across the y step
        constexpr bool PF = sizeof(T) == 4;
        if constexpr (PF) {
            load_src(pl);
            __builtin_amdgcn_s_waitcnt(0x0f70);  // nothing outstanding on entry to the loop (vmcnt 0)
        }
        for (;;) {
            lanes();
            if constexpr (!PF) load_src(pl);
            const PlaneRef r = plane_ref(args, pl);
            const uint32_t rs = rs_of(r);                                     // W row stride (bytes)
            const uint32_t wy_off = static_cast<uint32_t>(2 * yt) * rs + yc * CSZ;  // W row 2*yt, column yc
            cx<T> *Wz = W_of(r);
            cx<T> *Wnz = Wn_of(r);
            {  // x step
                cx<T> v[E];
#pragma unroll
                for (int m = 0; m < E; ++m) v[m] = m < H ? s[m] : cx<T>{T(0), T(0)};
                // no leading barrier: the end of the previous plane has one
                RowF::template run<K, false>(v, ax, lds, SP, twl, xc, xt);
                // X[k] = (U[k] + U*[n-k])/2 - (i/2) exp(-i pi k/n) (U[k] - U*[n-k]); the
                // partners U[n-k] come from the mirror lane of the row
                cx<T> wp[E];
                mirror_partners<T, E, NB>(v, wp, xt, tid & 63);
                if constexpr (K == 1) __syncthreads();  // post table visible
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int k = xt + NB * m;
                    const cx<T> u = v[m];
                    const cx<T> w = wp[m];
                    const cx<T> a = {static_cast<T>(0.5) * (u.x + w.x), static_cast<T>(0.5) * (u.y - w.y)};
                    const cx<T> b = {static_cast<T>(0.5) * (u.x - w.x), static_cast<T>(0.5) * (u.y + w.y)};
                    const cx<T> eb = cmul(post[k], b);
                    v[m] = cx<T>{a.x + eb.y, a.y - eb.x};
                    if (m == 0 && xt == 0) v[m].y = u.x - u.y;  // X[0] is real: its imaginary slot takes X[n]
                }
                // to the row: each thread writes the positions its last gather read
                cx<T> *row = lds + xc * SP;
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int P = xt + NB * m;
                    row[P + (P >> 4)] = v[m];
                }
            }
            __syncthreads();
            const int nxt = pl + G;
            {  // y step
                // w, the odd half's input x[y] e^{-i pi y/n}, is formed after the even
                // transform from a copy of the column: formed up front, the two halves
                // and the factors do not fit the 128 registers of a 1024-thread group
                cx<T> v[E], w[E];
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int y = yt + NB * m;
                    v[m] = lds[y * SP + cp];
                    w[m] = v[m];
                }
                // The next source plane, before this plane's stores: loads and
                // stores retire in order, so a load issued after them could not be
                // waited for without waiting for them.
                if constexpr (PF) {
                    if (nxt < args.nwg) load_src(nxt);
                }
                // Column 0 carries C = A + i B, A and B the transforms of the real
                // columns kx = 0 and kx = n: A[ky] = (C[ky] + conj C[-ky])/2 goes to
                // W and B[ky] = (C[ky] - conj C[-ky])/(2i) to the Nyquist column.
                // Its threads are lanes of wavefront 0, so the partners C[-ky] come
                // from other lanes: position (n - j) mod n of the even half (the
                // mirror lane, as in the split step) and n - 1 - j of the odd half.
                auto emit = [&](const cx<T> *q, const int parity) {
                    if (tid < 64) {
                        const bool col0 = yc == 0;
                        const int lane = tid;
                        const int addr = parity == 0 ? (lane - yt + ((NB - yt) & (NB - 1))) << 2
                                                     : (lane - yt + (NB - 1 - yt)) << 2;
#pragma unroll
                        for (int m = 0; m < E; ++m) {
                            // every lane sends position E-1-m; thread 0's even partner is its
                            // own register (E - m) mod E
                            const cx<T> d = q[E - 1 - m];
                            cx<T> Cp = {lane_read(addr, d.x), lane_read(addr, d.y)};
                            if (parity == 0 && yt == 0) Cp = q[(E - m) % E];
                            const cx<T> C = q[m];
                            const cx<T> A = {static_cast<T>(0.5) * (C.x + Cp.x), static_cast<T>(0.5) * (C.y - Cp.y)};
                            const cx<T> B = {static_cast<T>(0.5) * (C.y + Cp.y), static_cast<T>(-0.5) * (C.x - Cp.x)};
                            const cx<T> o = {col0 ? A.x : C.x, col0 ? A.y : C.y};  // by value: C stays in registers
                            at<T>(Wz, wy_off + (m * 2 * NB + parity) * rs) = o;
                            if (col0) Wnz[2 * (yt + NB * m) + parity] = B;
                        }
                    } else {
#pragma unroll
                        for (int m = 0; m < E; ++m) at<T>(Wz, wy_off + (m * 2 * NB + parity) * rs) = q[m];
                    }
                };
                ColF::template run<K>(v, ax, lds, SP, twl, cp, yt);  // Y[2j]
                emit(v, 0);
#pragma unroll
                for (int m = 0; m < E; ++m) w[m] = cmul(w[m], post[yt + NB * m]);
                ColF::template run<K>(w, ax, lds, SP, twl, cp, yt);  // Y[2j+1]
                emit(w, 1);
            }
            if (nxt >= args.nwg) break;
            pl = nxt;
            __syncthreads();  // LDS readers of this plane are done
        }
    } else {
        cx<T> *sep = twl + (2 * n - 1);
        constexpr int NWV = (2 * n + BLK - 1) / BLK;  // Nyquist values per thread
        cx<T> e[E];     // even W rows of this thread's column, current plane
        cx<T> nw[NWV];  // Nyquist column of the next plane, on its way to `sep`
        // The Nyquist values are loaded first, so that waiting for them leaves the
        // even rows in flight.
        auto load_even = [&](int p) {
            const PlaneRef r = plane_ref(args, p);
            const cx<T> *Wz = W_of(r);
            const cx<T> *Wnz = Wn_of(r);
            const uint32_t rs = rs_of(r);
            const uint32_t even_off = static_cast<uint32_t>(2 * yt) * rs + yc * CSZ;
#pragma unroll
            for (int q = 0; q < NWV; ++q) {  // clamped, so every thread loads (no divergent definition)
                const int i = tid + q * BLK;
                if constexpr (NT) nw[q] = ld_nt(&Wnz[i < 2 * n ? i : 2 * n - 1]);
                else nw[q] = Wnz[i < 2 * n ? i : 2 * n - 1];
            }
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if constexpr (NT) e[m] = ld_nt(&at<T>(Wz, even_off + m * 2 * NB * rs));
                else e[m] = at<T>(Wz, even_off + m * 2 * NB * rs);
            }
        };
        auto stage_nyquist = [&]() {
#pragma unroll
            for (int q = 0; q < NWV; ++q) {
                const int i = tid + q * BLK;
                if (i < 2 * n) sep[i] = nw[q];
            }
        };
        load_even(pl);
        stage_nyquist();
        __syncthreads();  // twiddles and the first Nyquist column visible
        // One plane; false after the workgroup's last.  The first plane is a copy
        // of its own, so that every entry to the loop follows a plane's stores:
        // the compiler then counts those stores in its wait for the prefetched
        // even rows, instead of draining them there (entered from the prologue,
        // which stores nothing, the loop's waits assumed no stores in flight).
        auto one_plane = [&]() __attribute__((always_inline)) -> bool {
            lanes();
            const PlaneRef r = plane_ref(args, pl);
            const uint32_t rs = rs_of(r);
            const uint32_t even_off = static_cast<uint32_t>(2 * yt) * rs + yc * CSZ;
            const cx<T> *Wz = W_of(r);
            cx<T> o[E];  // odd rows, in flight while the even ones are transformed
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if constexpr (NT) o[m] = ld_nt(&at<T>(Wz, even_off + (m * 2 * NB + 1) * rs));
                else o[m] = at<T>(Wz, even_off + (m * 2 * NB + 1) * rs);
            }
            // the barrier before the loop or at the end of the previous plane
            // published the Nyquist column and retired the readers of the plane
            {  // y step: column kx = 0 also carries kx = n (as Y0 + i Yn)
                if (yc == 0) {
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const cx<T> a = sep[2 * (yt + NB * m)];
                        e[m] = cx<T>{e[m].x - a.y, e[m].y + a.x};
                    }
                }
                ColI::template run<K, false>(e, ax, lds, SP, twl, cp, yt);
                if (yc == 0) {
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const cx<T> b = sep[2 * (yt + NB * m) + 1];
                        o[m] = cx<T>{o[m].x - b.y, o[m].y + b.x};
                    }
                }
                ColI::template run<K>(o, ax, lds, SP, twl, cp, yt);
                // x[y] = A[y] + e^{+i pi y/n} B[y]; each thread writes the positions its last gather read
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int y = yt + NB * m;
                    lds[y * SP + cp] = e[m] + cmulc(o[m], post[y]);
                }
            }
            __syncthreads();
            const int nxt = pl + G;
            if (nxt < args.nwg) load_even(nxt);
            {  // x step
                const cx<T> *row = lds + xc * SP;
                const cx<T> p0 = row[0];  // X[y][0] + i X[y][n], both real
                cx<T> v[E];
                // U[k] = (X[k] + X*[n-k]) + i exp(+i pi k/n) (X[k] - X*[n-k])
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int k = xt + NB * m;
                    cx<T> a, b;
                    if (m == 0 && xt == 0) {
                        a = cx<T>{p0.x, T(0)};
                        b = cx<T>{p0.y, T(0)};
                    } else {
                        const int kp = n - k;
                        a = row[k + (k >> 4)];
                        b = row[kp + (kp >> 4)];
                    }
                    const cx<T> sm = {a.x + b.x, a.y - b.y};
                    const cx<T> df = {a.x - b.x, a.y + b.y};
                    const cx<T> ed = cmulc(df, post[k]);
                    v[m] = cx<T>{sm.x - ed.y, sm.y + ed.x};
                }
                RowI::template run<K>(v, ax, lds, SP, twl, xc, xt);
                void *plane = static_cast<T *>(r.pa->Phi) + static_cast<size_t>(r.z) * n * n;
                const uint32_t off = static_cast<uint32_t>((xc * n + 2 * xt) * sizeof(T));
#pragma unroll
                for (int m = 0; m < H; ++m) at<T>(plane, off + m * NB * CSZ) = v[m];
            }
            if (nxt < args.nwg) stage_nyquist();  // `sep` is free until the next y step
            if (nxt >= args.nwg) return false;
            pl = nxt;
            __syncthreads();  // LDS readers of this plane are done
            return true;
        };
        if (one_plane())
            while (one_plane()) {
            }
    }
}

// Planes one workgroup of a plane kernel takes at most (PSPFFT_PLANES_PER_WG,
// default 8).
inline int planes_per_workgroup() {
    static int v = 0;
    if (v == 0) {
        const char *e = std::getenv("PSPFFT_PLANES_PER_WG");
        const int x = e ? std::atoi(e) : 0;
        v = x >= 1 && x <= 1024 ? x : 8;
    }
    return v;
}

// Grid: a whole number of generations of what the device holds at once (from
// the occupancy of this kernel), as few as keep every workgroup at or below
// planes_per_workgroup() planes; never more than one per plane.
template <typename T, int E, int K, bool FWD>
hipError_t launch_plane_kernel(const LaunchArgs &args, size_t lds, hipStream_t stream) {
    constexpr int kMaxDevices = 64;
    static int resident[kMaxDevices] = {0};
    auto fn = plane_kernel<T, E, K, FWD>;
    // inverse planes of a streaming launch: nontemporal row loads
    auto fs = plane_kernel<T, E, K, FWD, !FWD>;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (resident[dev] == 0) {
        for (auto f : {fn, fs}) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    160 * 1024);
            if (e != hipSuccess) return e;
        }
        int per_cu = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, E * K * K, lds);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        resident[dev] = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    }
    // at most planes_per_workgroup() planes each: more workgroups than the device
    // holds at once leave room for kernels on other streams
    // whole generations of resident workgroups, each taking at most `per` planes:
    // workgroups then differ by at most one plane, and no short last generation
    // runs alone at the end
    const int per = planes_per_workgroup();
    const long gens = (static_cast<long>(args.nwg) + static_cast<long>(resident[dev]) * per - 1) /
                      (static_cast<long>(resident[dev]) * per);
    int grid = static_cast<int>(gens * resident[dev]);
    if (grid > args.nwg) grid = args.nwg;
    hipLaunchKernelGGL(args.nt ? fs : fn, dim3(grid), dim3(E * K * K), lds, stream, args);
    return hipGetLastError();
}

template <typename T, int E, int K>
hipError_t launch_plane_k(bool fwd, const LaunchArgs &args, int grid, size_t lds, hipStream_t stream) {
    constexpr int prec = sizeof(T) == 4 ? 0 : 1;
    if constexpr (plane_fits(prec, E, K)) {
        if (lds != plane_lds_bytes(prec, E, K)) return hipErrorInvalidValue;
        return fwd ? launch_plane_kernel<T, E, K, true>(args, lds, stream)
                   : launch_plane_kernel<T, E, K, false>(args, lds, stream);
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T, int E>
hipError_t launch_plane_family(bool fwd, int K, const LaunchArgs &args, int grid, size_t lds, hipStream_t stream) {
    switch (K) {
        case 1: return launch_plane_k<T, E, 1>(fwd, args, grid, lds, stream);
        case 2: return launch_plane_k<T, E, 2>(fwd, args, grid, lds, stream);
        case 4: return launch_plane_k<T, E, 4>(fwd, args, grid, lds, stream);
        case 8: return launch_plane_k<T, E, 8>(fwd, args, grid, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pspfft

// One translation unit per (precision, family) keeps compiles parallel.
#define PSPFFT_FAMILY(T, E, NAME, PLANE)                                                            \
    namespace pspfft {                                                                              \
    hipError_t NAME(int mode, int K, int fix, const LaunchArgs &args, int grid, int block,          \
                    size_t lds, hipStream_t stream) {                                               \
        return launch_family<T, E>(mode, K, fix, args, grid, block, lds, stream);                   \
    }                                                                                               \
    hipError_t PLANE(bool fwd, int K, const LaunchArgs &args, int grid, size_t lds, hipStream_t stream) { \
        return launch_plane_family<T, E>(fwd, K, args, grid, lds, stream);                          \
    }                                                                                               \
    }
