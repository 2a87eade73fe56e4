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
//            C of X0 + i Xn; one wave separates the two real columns at the end
//            with A[k] = (C[k] + conj C[-k])/2 and B[k] = (C[k] - conj C[-k])/(2i).
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

#include "pass_kernels.h"

namespace pspfft {

template <typename T, int E, int K, bool FWD>
__global__ void __launch_bounds__(E * K * K) plane_kernel(const LaunchArgs args) {
    constexpr int n = E * K;
    constexpr int NB = K;
    constexpr int H = E / 2;
    constexpr int CSZ = static_cast<int>(sizeof(cx<T>));
    constexpr int SP = row_stride(n, NB, CSZ);  // LDS row stride of the plane
    using RowF = LineFFT<T, E, -1, true, NB, SP>;
    using RowI = LineFFT<T, E, +1, true, NB, SP>;
    using ColF = LineFFT<T, E, -1, false, NB, SP>;
    using ColI = LineFFT<T, E, +1, false, NB, SP>;

    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem);

    const int bid = static_cast<int>(blockIdx.x);
    if (bid >= args.nwg) return;
    int sgi = 0;
    while (sgi + 1 < args.nseg && bid >= args.seg[sgi + 1].wg_begin) ++sgi;
    const Segment &sg = args.seg[sgi];
    const int local = bid - sg.wg_begin;
    const int member = local % sg.group;
    const int z = local / sg.group;
    const ProbArg &pa = args.p[sg.first + member];
    const AxisPlan &ax = pa.plan->ax[0];

    // stage twiddles (n - 1 entries), exp(-i pi k / n) (k < n), and 2n slots
    // for column 0 of the forward y step
    cx<T> *twl = lds + n * SP;
    const cx<T> *post = twl + (n - 1);
    cx<T> *sep = twl + (2 * n - 1);
    copy_to_lds<T>(twl, ax.tw, 2 * n - 1);

    const int tid = static_cast<int>(threadIdx.x);
    cx<T> *Wz = static_cast<cx<T> *>(pa.W) + static_cast<size_t>(z) * 2 * n * n;
    cx<T> *Wnz = static_cast<cx<T> *>(pa.Wn) + static_cast<size_t>(z) * 2 * n;

    if constexpr (FWD) {
        {  // x step: row c = y, thread t of the row
            const int c = tid / NB, t = tid % NB;
            cx<T> v[E];
            const cx<T> *src =
                reinterpret_cast<const cx<T> *>(static_cast<const T *>(pa.S) + (static_cast<size_t>(z) * n + c) * n) + t;
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = m < H ? src[NB * m] : cx<T>{T(0), T(0)};
            RowF::template run<K>(v, ax, lds, SP, twl, c, t);
            // U[k] to the row (each thread writes the positions its last gather read)
            cx<T> *row = lds + c * SP;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int P = t + NB * m;
                row[P + (P >> 4)] = v[m];
            }
            __syncthreads();
            // X[k] = (U[k] + U*[n-k])/2 - (i/2) exp(-i pi k/n) (U[k] - U*[n-k])
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int k = t + NB * m;
                const int kp = k == 0 ? 0 : n - k;
                const cx<T> u = v[m];
                const cx<T> w = row[kp + (kp >> 4)];
                const cx<T> a = {static_cast<T>(0.5) * (u.x + w.x), static_cast<T>(0.5) * (u.y - w.y)};
                const cx<T> b = {static_cast<T>(0.5) * (u.x - w.x), static_cast<T>(0.5) * (u.y + w.y)};
                const cx<T> eb = cmul(post[k], b);
                v[m] = cx<T>{a.x + eb.y, a.y - eb.x};
                if (m == 0 && t == 0) v[m].y = u.x - u.y;  // X[0] is real: its imaginary slot takes X[n]
            }
            __syncthreads();  // partner reads done
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int P = t + NB * m;
                row[P + (P >> 4)] = v[m];
            }
        }
        __syncthreads();
        {  // y step: column c = kx, thread t of the column
            const int c = tid % n, t = tid / n;
            const int cp = c + (c >> 4);
            cx<T> v[E], w[E];
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int y = t + NB * m;
                v[m] = lds[y * SP + cp];
                w[m] = cmul(v[m], post[y]);
            }
            // Column 0 parks its values in `sep`; the other columns go straight to W.
            auto emit = [&](const cx<T> *r, const int parity) {
                if (c == 0) {
#pragma unroll
                    for (int m = 0; m < E; ++m) sep[2 * (t + NB * m) + parity] = r[m];
                } else {
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const int ky = 2 * (t + NB * m) + parity;
                        Wz[static_cast<size_t>(ky) * n + c] = r[m];
                    }
                }
            };
            ColF::template run<K>(v, ax, lds, SP, twl, cp, t);  // Y[2j]
            emit(v, 0);
            ColF::template run<K>(w, ax, lds, SP, twl, cp, t);  // Y[2j+1]
            emit(w, 1);
        }
        __syncthreads();
        // The first wave separates column 0: C = A + i B with A, B the transforms
        // of the real columns kx = 0 and kx = n.
        constexpr int NT = E * K * K < 64 ? E * K * K : 64;
        if (tid < NT) {
            for (int ky = tid; ky < 2 * n; ky += NT) {
                const int kp = ky == 0 ? 0 : 2 * n - ky;
                const cx<T> C = sep[ky];
                const cx<T> Cp = sep[kp];
                Wz[static_cast<size_t>(ky) * n] =
                    cx<T>{static_cast<T>(0.5) * (C.x + Cp.x), static_cast<T>(0.5) * (C.y - Cp.y)};
                Wnz[ky] = cx<T>{static_cast<T>(0.5) * (C.y + Cp.y), static_cast<T>(-0.5) * (C.x - Cp.x)};
            }
        }
    } else {
        {  // y step: column c = kx (kx = 0 also carries kx = n), thread t
            const int c = tid % n, t = tid / n;
            const int cp = c + (c >> 4);
            cx<T> v[E], w[E];
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int j = t + NB * m;
                v[m] = Wz[static_cast<size_t>(2 * j) * n + c];
                w[m] = Wz[static_cast<size_t>(2 * j + 1) * n + c];
            }
            if (c == 0) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int j = t + NB * m;
                    const cx<T> a = Wnz[2 * j], b = Wnz[2 * j + 1];
                    v[m] = cx<T>{v[m].x - a.y, v[m].y + a.x};
                    w[m] = cx<T>{w[m].x - b.y, w[m].y + b.x};
                }
            }
            ColI::template run<K>(v, ax, lds, SP, twl, cp, t);
            ColI::template run<K>(w, ax, lds, SP, twl, cp, t);
            if constexpr (K == 1) __syncthreads();  // post table visible
            // x[y] = A[y] + e^{+i pi y/n} B[y]; each thread writes the positions its last gather read
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int y = t + NB * m;
                lds[y * SP + cp] = v[m] + cmulc(w[m], post[y]);
            }
        }
        __syncthreads();
        {  // x step: row c = y, thread t
            const int c = tid / NB, t = tid % NB;
            const cx<T> *row = lds + c * SP;
            const cx<T> p0 = row[0];  // X[y][0] + i X[y][n], both real
            cx<T> v[E];
            // U[k] = (X[k] + X*[n-k]) + i exp(+i pi k/n) (X[k] - X*[n-k])
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int k = t + NB * m;
                cx<T> a, b;
                if (m == 0 && t == 0) {
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
            RowI::template run<K>(v, ax, lds, SP, twl, c, t);
            cx<T> *dst =
                reinterpret_cast<cx<T> *>(static_cast<T *>(pa.Phi) + (static_cast<size_t>(z) * n + c) * n) + t;
#pragma unroll
            for (int m = 0; m < H; ++m) dst[NB * m] = v[m];
        }
    }
}

template <typename T, int E, int K, bool FWD>
hipError_t launch_plane_kernel(const LaunchArgs &args, int grid, size_t lds, hipStream_t stream) {
    static bool attr_set = false;
    auto fn = plane_kernel<T, E, K, FWD>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(E * K * K), lds, stream, args);
    return hipGetLastError();
}

template <typename T, int E, int K>
hipError_t launch_plane_k(bool fwd, const LaunchArgs &args, int grid, size_t lds, hipStream_t stream) {
    constexpr int prec = sizeof(T) == 4 ? 0 : 1;
    if constexpr (plane_fits(prec, E, K)) {
        if (lds != plane_lds_bytes(prec, E, K)) return hipErrorInvalidValue;
        return fwd ? launch_plane_kernel<T, E, K, true>(args, grid, lds, stream)
                   : launch_plane_kernel<T, E, K, false>(args, grid, lds, stream);
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
    hipError_t NAME(int mode, int K, bool fix, const LaunchArgs &args, int grid, int block,         \
                    size_t lds, hipStream_t stream) {                                               \
        return launch_family<T, E>(mode, K, fix, args, grid, block, lds, stream);                   \
    }                                                                                               \
    hipError_t PLANE(bool fwd, int K, const LaunchArgs &args, int grid, size_t lds, hipStream_t stream) { \
        return launch_plane_family<T, E>(fwd, K, args, grid, lds, stream);                          \
    }                                                                                               \
    }
