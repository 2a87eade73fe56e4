// pspfft_kernels.hip -- gfx950 kernels for the mesh-doubling Poisson solve
// (Budiardja & Cardall, arXiv:1106.0557, Sec. 2.1 and 2.2.2).
//
// One solve is five streaming passes over the workspace (layout in internal.h):
//   X_FWD  : rows of S, zero-padded to 2nx, transformed along x (Sec. 2.2.2, x pillars)
//   Y_FWD  : columns along y; the input half y >= ny is known zero and never read
//   Z_CONV : columns along z: forward transform (input half zero), multiply by the
//            Green's-function spectrum, inverse transform, keep z < nz (Sec. 2.1, the
//            convolution theorem; Sec. 2.2.2, the multiply happens in z pillars)
//   Y_INV  : inverse along y, keep y < ny
//   X_INV  : inverse along x with the Hermitian extension, keep x < nx -> Phi
// The normalisation 1/((2nx)(2ny)(2nz)) is folded into the spectrum.
//
// Line FFT engine.  A line of length L = 2n is owned by NB = L/E threads of one
// workgroup; thread t holds positions t + NB*m (m < E) in registers.  Each stage
// of radix R applies E/R radix-R butterflies per thread (Stockham, decimation in
// time, twiddles from an FP64-generated table), scattering to LDS; the next stage
// gathers the thread's own positions back.  The first stage reads straight from
// global memory and the last stage leaves the result in registers, so a 2-stage
// line costs one LDS exchange.  A workgroup holds TILE = blockDim / NB lines that
// are adjacent in memory (consecutive kx for the column passes), so every
// global access of a wavefront is a few full 128-byte segments.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "internal.h"

namespace pspfft {

// ------------------------------------------------------------ complex math --

template <typename T>
struct cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.x * s, a.y * s}; }

// ------------------------------------------- compile-time trigonometry --
// cos and sin of 2 pi num/den, evaluated by the compiler: the rational angle is
// folded into [0, pi/4] by exact integer symmetry steps and the Taylor series is
// summed in double precision (error well below one float ulp).

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double series_sin(double x) {
    double term = x, sum = x;
    for (int i = 1; i < 16; ++i) {
        term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}

constexpr double series_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int i = 1; i < 16; ++i) {
        term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}

struct CosSin {
    double c, s;
};

constexpr CosSin turn(long num, long den) {
    num %= den;
    if (num < 0) num += den;
    bool neg_s = false, neg_c = false, swap = false;
    if (2 * num > den) {  // q -> 1 - q
        num = den - num;
        neg_s = true;
    }
    if (4 * num > den) {  // q -> 1/2 - q
        num = den - 2 * num;
        den *= 2;
        neg_c = true;
    }
    if (8 * num > den) {  // q -> 1/4 - q
        num = den - 4 * num;
        den *= 4;
        swap = true;
    }
    const double x = 2.0 * kPi * static_cast<double>(num) / static_cast<double>(den);
    double c = series_cos(x), s = series_sin(x);
    if (swap) {
        const double t = c;
        c = s;
        s = t;
    }
    if (neg_c) c = -c;
    if (neg_s) s = -s;
    return {c, s};
}

template <int I, int N, typename F>
__device__ __forceinline__ void sfor(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        sfor<I + 1, N>(f);
    }
}

// a * exp(DIR 2 pi i e / R) with e, R known at compile time.
template <int R, int DIR, int e, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> a) {
    constexpr int em = ((e % R) + R) % R;
    if constexpr (em == 0) {
        return a;
    } else if constexpr (2 * em == R) {
        return {-a.x, -a.y};
    } else if constexpr (4 * em == R) {  // DIR * i
        if constexpr (DIR > 0) return {-a.y, a.x};
        else return {a.y, -a.x};
    } else if constexpr (4 * em == 3 * R) {  // -DIR * i
        if constexpr (DIR > 0) return {a.y, -a.x};
        else return {-a.y, a.x};
    } else {
        constexpr CosSin w = turn(static_cast<long>(DIR) * em, R);
        const T c = static_cast<T>(w.c), s = static_cast<T>(w.s);
        return {a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

constexpr int first_factor(int R) {
    if (R % 4 == 0 && R > 4) return 4;
    for (int p = 2; p <= R; ++p)
        if (R % p == 0) return p;
    return R;
}

// In-register DFT of length R, natural order in and out:
// X[k] = sum_j x[j] exp(DIR 2 pi i j k / R).
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T> *x) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        const cx<T> a = x[0], b = x[1];
        x[0] = a + b;
        x[1] = a - b;
    } else if constexpr (R == 3) {
        constexpr T h = static_cast<T>(0.8660254037844386467637231707529362);  // sin(2 pi / 3)
        const cx<T> s = x[1] + x[2], d = x[1] - x[2];
        const cx<T> m = {x[0].x - static_cast<T>(0.5) * s.x, x[0].y - static_cast<T>(0.5) * s.y};
        // DIR * i * h * d
        const cx<T> n = DIR > 0 ? cx<T>{-h * d.y, h * d.x} : cx<T>{h * d.y, -h * d.x};
        x[0] = x[0] + s;
        x[1] = m + n;
        x[2] = m - n;
    } else if constexpr (R == 4) {
        const cx<T> t0 = x[0] + x[2], t1 = x[0] - x[2], t2 = x[1] + x[3];
        const cx<T> t3 = rot<4, DIR, 1>(x[1] - x[3]);
        x[0] = t0 + t2;
        x[2] = t0 - t2;
        x[1] = t1 + t3;
        x[3] = t1 - t3;
    } else if constexpr (R == 5) {
        constexpr CosSin w1 = turn(1, 5), w2 = turn(2, 5);
        const T c1 = static_cast<T>(w1.c), c2 = static_cast<T>(w2.c);
        const T s1 = static_cast<T>(w1.s), s2 = static_cast<T>(w2.s);
        const cx<T> a1 = x[1] + x[4], d1 = x[1] - x[4], a2 = x[2] + x[3], d2 = x[2] - x[3];
        const cx<T> p1 = {x[0].x + c1 * a1.x + c2 * a2.x, x[0].y + c1 * a1.y + c2 * a2.y};
        const cx<T> p2 = {x[0].x + c2 * a1.x + c1 * a2.x, x[0].y + c2 * a1.y + c1 * a2.y};
        const cx<T> u1 = {s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y};
        const cx<T> u2 = {s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y};
        // q = DIR * i * u
        const cx<T> q1 = DIR > 0 ? cx<T>{-u1.y, u1.x} : cx<T>{u1.y, -u1.x};
        const cx<T> q2 = DIR > 0 ? cx<T>{-u2.y, u2.x} : cx<T>{u2.y, -u2.x};
        x[0] = x[0] + a1 + a2;
        x[1] = p1 + q1;
        x[4] = p1 - q1;
        x[2] = p2 + q2;
        x[3] = p2 - q2;
    } else {
        // Cooley-Tukey in registers, R = P * Q, input index q + Q p, output k1 + P k2.
        constexpr int P = first_factor(R);
        constexpr int Q = R / P;
        cx<T> a[P][Q];
        sfor<0, Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            cx<T> u[P];
            sfor<0, P>([&](auto pc) {
                constexpr int p = decltype(pc)::value;
                u[p] = x[q + Q * p];
            });
            dft<P, DIR>(u);
            sfor<0, P>([&](auto kc) {
                constexpr int k1 = decltype(kc)::value;
                a[k1][q] = rot<R, DIR, q * k1>(u[k1]);
            });
        });
        sfor<0, P>([&](auto kc) {
            constexpr int k1 = decltype(kc)::value;
            dft<Q, DIR>(a[k1]);
            sfor<0, Q>([&](auto k2c) {
                constexpr int k2 = decltype(k2c)::value;
                x[k1 + P * k2] = a[k1][k2];
            });
        });
    }
}

// -------------------------------------------------------------- the engine --

template <typename T, int E, int DIR>
struct LineFFT {
    // One stage of radix R on the thread's E registers (E/R butterflies).
    template <int R>
    static __device__ __forceinline__ void stage(cx<T> *v, const AxisPlan &ax, int s, bool last, cx<T> *lds,
                                                 int ldsw, int c, int t) {
        constexpr int NBF = E / R;
        const int NB = ax.NB;
        const int Ns = ax.Ns[s];
        const uint32_t mg = ax.magic[s];
        const cx<T> *tw = static_cast<const cx<T> *>(ax.tw) + ax.twoff[s];
        if (!last) __syncthreads();  // earlier readers of LDS are done
        sfor<0, NBF>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const int b = t + NB * i;
            int q = b, k = 0;
            if (s > 0) {
                q = static_cast<int>(__umulhi(static_cast<uint32_t>(b), mg));
                k = b - q * Ns;
            }
            cx<T> x[R];
            sfor<0, R>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                x[r] = v[i + r * NBF];
            });
            if (s > 0) {
                const cx<T> *twk = tw + k * (R - 1);
                sfor<1, R>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    cx<T> w = twk[r - 1];
                    if constexpr (DIR > 0) w.y = -w.y;
                    x[r] = cmul(x[r], w);
                });
            }
            dft<R, DIR>(x);
            if (last) {
                sfor<0, R>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    v[i + r * NBF] = x[r];
                });
            } else {
                const int base = q * Ns * R + k;
                sfor<0, R>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    lds[(base + r * Ns) * ldsw + c] = x[r];
                });
            }
        });
    }

    static __device__ __forceinline__ void run(cx<T> *v, const AxisPlan &ax, cx<T> *lds, int ldsw, int c, int t) {
        const int NB = ax.NB;
        const int nst = ax.nst;
        for (int s = 0; s < nst; ++s) {
            const bool last = s == nst - 1;
            if (s > 0) {
                __syncthreads();
#pragma unroll
                for (int m = 0; m < E; ++m) v[m] = lds[(t + NB * m) * ldsw + c];
            }
            const int R = ax.R[s];
            if (R == E) {
                stage<E>(v, ax, s, last, lds, ldsw, c, t);
            } else if (R == 8) {
                if constexpr (E % 8 == 0 && E != 8) stage<8>(v, ax, s, last, lds, ldsw, c, t);
            } else if (R == 4) {
                if constexpr (E % 4 == 0 && E != 4) stage<4>(v, ax, s, last, lds, ldsw, c, t);
            } else if (R == 2) {
                if constexpr (E % 2 == 0 && E != 2) stage<2>(v, ax, s, last, lds, ldsw, c, t);
            }
        }
    }
};

// ------------------------------------------------------------ pass kernels --

// Largest workgroup per (precision, radix family), chosen so that the E
// registers per thread fit without spilling.
template <typename T, int E>
constexpr int kMaxBlock = (sizeof(T) == 4) ? (E == 16 ? 1024 : (E <= 24 ? 512 : 256)) : (E == 16 ? 512 : 256);

template <typename T, int E, int MODE>
__global__ void __launch_bounds__((kMaxBlock<T, E>)) pass_kernel(const LaunchArgs args) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem);

    const int bid = blockIdx.x;
    int p = 0;
    while (p + 1 < args.count && bid >= args.p[p + 1].wg_begin) ++p;
    const ProbArg &pa = args.p[p];
    const DevPlan &pl = *pa.plan;
    constexpr int axis = (MODE == X_FWD || MODE == X_INV) ? 0 : (MODE == Z_CONV ? 2 : 1);
    const AxisPlan &ax = pl.ax[axis];
    const int nx = pl.nx, ny = pl.ny, nz = pl.nz;
    const int NB = ax.NB;
    const int L = ax.L;
    const int tile = static_cast<int>(blockDim.x) / NB;  // lines per workgroup (power of two)
    const int tshift = __builtin_ctz(tile);
    const int tid = threadIdx.x;
    const int c = tid & (tile - 1);
    const int t = tid >> tshift;
    const int ldsw = tile;

    int local = bid - pa.wg_begin;
    const bool nyq = local >= pa.wg_main;
    if (nyq) local -= pa.wg_main;
    const int g = local * tile + c;  // line index within its set

    cx<T> v[E];
    cx<T> *W = static_cast<cx<T> *>(pa.W);
    cx<T> *Wn = static_cast<cx<T> *>(pa.Wn);

    if constexpr (MODE == X_FWD || MODE == X_INV) {
        // Lines are rows (y, z), y < ny, z < nz; row r = z*ny + y.
        const int nrows = ny * nz;
        const bool active = g < nrows;
        const int z = active ? g / ny : 0;
        const int y = g - z * ny;
        cx<T> *wrow = W + (static_cast<size_t>(z) * 2 * ny + y) * nx;
        cx<T> *wnyq = Wn + static_cast<size_t>(z) * 2 * ny + y;
        if constexpr (MODE == X_FWD) {
            const T *srow = static_cast<const T *>(pa.S) + static_cast<size_t>(g) * nx;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int P = t + NB * m;
                if (active && P < nx) v[m] = cx<T>{srow[P], T(0)};
                else v[m] = cx<T>{T(0), T(0)};
            }
            LineFFT<T, E, -1>::run(v, ax, lds, ldsw, c, t);
            if (active) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int P = t + NB * m;
                    if (P < nx) wrow[P] = v[m];
                    else if (P == nx) *wnyq = v[m];
                }
            }
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int P = t + NB * m;
                cx<T> a = {T(0), T(0)};
                if (active) {
                    if (P < nx) {
                        a = wrow[P];
                    } else if (P == nx) {
                        a = *wnyq;
                    } else {  // Hermitian extension: X[L - P] conjugated
                        const cx<T> b = wrow[L - P];
                        a = {b.x, -b.y};
                    }
                }
                v[m] = a;
            }
            LineFFT<T, E, +1>::run(v, ax, lds, ldsw, c, t);
            if (active) {
                T *prow = static_cast<T *>(pa.Phi) + static_cast<size_t>(g) * nx;
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int P = t + NB * m;
                    if (P < nx) prow[P] = v[m].x;
                }
            }
        }
    } else {
        // Column passes.  Line base and element stride of line g.
        cx<T> *base;
        size_t es;
        bool active;
        int ky = 0, kx = 0;
        if constexpr (MODE == Z_CONV) {
            if (!nyq) {
                active = g < 2 * ny * nx;
                ky = active ? g / nx : 0;
                kx = g - ky * nx;
                base = W + static_cast<size_t>(ky) * nx + kx;
                es = static_cast<size_t>(2) * ny * nx;
            } else {
                active = g < 2 * ny;
                ky = g;
                kx = nx;
                base = Wn + g;
                es = static_cast<size_t>(2) * ny;
            }
        } else {
            if (!nyq) {
                active = g < nz * nx;
                const int z = active ? g / nx : 0;
                kx = g - z * nx;
                base = W + static_cast<size_t>(z) * 2 * ny * nx + kx;
                es = nx;
            } else {
                active = g < nz;
                base = Wn + static_cast<size_t>(g) * 2 * ny;
                es = 1;
            }
        }
        const int nin = (MODE == Y_INV) ? L : (MODE == Z_CONV ? nz : ny);  // stored input rows
        const int nout = (MODE == Y_FWD) ? L : (MODE == Z_CONV ? nz : ny); // rows written back
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int P = t + NB * m;
            if (active && P < nin) v[m] = base[P * es];
            else v[m] = cx<T>{T(0), T(0)};
        }
        if constexpr (MODE == Y_FWD) {
            LineFFT<T, E, -1>::run(v, ax, lds, ldsw, c, t);
        } else if constexpr (MODE == Y_INV) {
            LineFFT<T, E, +1>::run(v, ax, lds, ldsw, c, t);
        } else {
            LineFFT<T, E, -1>::run(v, ax, lds, ldsw, c, t);
            // multiply by the spectrum, even in ky and kz: octant index min(k, 2n - k)
            const int kyo = ky <= ny ? ky : 2 * ny - ky;
            const T *Gp = nyq ? static_cast<const T *>(pl.Gn) + kyo
                              : static_cast<const T *>(pl.G) + static_cast<size_t>(kyo) * nx + kx;
            const size_t gs = nyq ? static_cast<size_t>(ny + 1) : static_cast<size_t>(ny + 1) * nx;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int P = t + NB * m;
                const int kzo = P <= nz ? P : L - P;
                const T gv = active ? Gp[kzo * gs] : T(0);
                v[m] = scale(v[m], gv);
            }
            LineFFT<T, E, +1>::run(v, ax, lds, ldsw, c, t);
        }
        if (active) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int P = t + NB * m;
                if (P < nout) base[P * es] = v[m];
            }
        }
    }
}

template <typename T, int E, int MODE>
static hipError_t launch_one(const LaunchArgs &args, int grid, int block, size_t lds, hipStream_t stream) {
    static bool attr_set = false;
    auto fn = pass_kernel<T, E, MODE>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, stream, args);
    return hipGetLastError();
}

template <typename T, int E>
static hipError_t launch_mode(int mode, const LaunchArgs &args, int grid, int block, size_t lds,
                              hipStream_t stream) {
    switch (mode) {
        case X_FWD: return launch_one<T, E, X_FWD>(args, grid, block, lds, stream);
        case Y_FWD: return launch_one<T, E, Y_FWD>(args, grid, block, lds, stream);
        case Z_CONV: return launch_one<T, E, Z_CONV>(args, grid, block, lds, stream);
        case Y_INV: return launch_one<T, E, Y_INV>(args, grid, block, lds, stream);
        case X_INV: return launch_one<T, E, X_INV>(args, grid, block, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_prec(int mode, int E, const LaunchArgs &args, int grid, int block, size_t lds,
                              hipStream_t stream) {
    switch (E) {
        case 16: return launch_mode<T, 16>(mode, args, grid, block, lds, stream);
        case 20: return launch_mode<T, 20>(mode, args, grid, block, lds, stream);
        case 24: return launch_mode<T, 24>(mode, args, grid, block, lds, stream);
        case 36: return launch_mode<T, 36>(mode, args, grid, block, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass(int mode, int prec, int E, const LaunchArgs &args, int grid, int block, size_t lds_bytes,
                       hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    return prec == 0 ? launch_prec<float>(mode, E, args, grid, block, lds_bytes, stream)
                     : launch_prec<double>(mode, E, args, grid, block, lds_bytes, stream);
}

int max_block(int prec, int E) {
    switch (E) {
        case 16: return prec == 0 ? kMaxBlock<float, 16> : kMaxBlock<double, 16>;
        case 20: return prec == 0 ? kMaxBlock<float, 20> : kMaxBlock<double, 20>;
        case 24: return prec == 0 ? kMaxBlock<float, 24> : kMaxBlock<double, 24>;
        default: return prec == 0 ? kMaxBlock<float, 36> : kMaxBlock<double, 36>;
    }
}

// ------------------------------------------ Green's-function spectrum (FP64) --

// Octant of Eq. (greens2) at integer offsets with the self-cell value of
// Eq. (greens_function): a[(r*(ny+1) + q)*(nx+1) + p], 0 <= p <= nx etc.
__global__ void green_fill(int nx, int ny, int nz, double hx, double hy, double hz, double *a) {
    const long total = static_cast<long>(nx + 1) * (ny + 1) * (nz + 1);
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const long p = i % (nx + 1);
    const long rest = i / (nx + 1);
    const long q = rest % (ny + 1);
    const long r = rest / (ny + 1);
    const double vol = hx * hy * hz;
    double v;
    if (p == 0 && q == 0 && r == 0) {
        const double hmin = fmin(hx, fmin(hy, hz));
        v = -vol / (4.0 * kPi * hmin);
    } else {
        const double dx = hx * p, dy = hy * q, dz = hz * r;
        v = -vol / (4.0 * kPi * sqrt(dx * dx + dy * dy + dz * dz));
    }
    a[i] = v;
}

// Transform of an even sequence of period 2n along one axis, evaluated on its
// n+1 independent values: out[k] = sum_{p=0}^{n} w_p in[p] cos(pi p k / n) with
// w_0 = w_n = 1 and w_p = 2 otherwise (the period-2n DFT of the mirrored line).
// The array is viewed as [A][M][B] with M = n+1 along the axis; a workgroup
// transforms `tw` lines that are adjacent in memory.
__global__ void green_axis(const double *in, double *out, int A, int M, int B, int tw,
                           const double *cos_tab /* cos(pi j / n), j < 2n */) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *line = reinterpret_cast<double *>(smem);  // [M][tw]
    const int n = M - 1;
    double *ct = line + static_cast<size_t>(M) * tw;  // [2n]
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int j = tid; j < 2 * n; j += nt) ct[j] = cos_tab[j];
    // lines of this workgroup: (a, b0 .. b0+tw) when B > 1, or (a0 .. a0+tw) when B == 1
    const long blk = blockIdx.x;
    long a0, b0;
    if (B > 1) {
        const long nbt = (B + tw - 1) / tw;
        a0 = blk / nbt;
        b0 = (blk % nbt) * tw;
    } else {
        a0 = blk * tw;
        b0 = 0;
    }
    auto addr = [&](int l, int m) -> long {
        return B > 1 ? (a0 * M + m) * static_cast<long>(B) + b0 + l : ((a0 + l) * M + m);
    };
    auto valid = [&](int l) -> bool { return B > 1 ? (b0 + l < B) : (a0 + l < A); };
    for (int e = tid; e < M * tw; e += nt) {
        int l, m;
        if (B > 1) {
            l = e % tw;
            m = e / tw;
        } else {
            m = e % M;
            l = e / M;
        }
        line[m * tw + l] = valid(l) ? in[addr(l, m)] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < M * tw; e += nt) {
        int l, k;
        if (B > 1) {
            l = e % tw;
            k = e / tw;
        } else {
            k = e % M;
            l = e / M;
        }
        double acc = line[l] + ((k & 1) ? -line[n * tw + l] : line[n * tw + l]);
        int j = k;  // (p * k) mod 2n
        double acc2 = 0.0;
        for (int p = 1; p < n; ++p) {
            acc2 += line[p * tw + l] * ct[j];
            j += k;
            if (j >= 2 * n) j -= 2 * n;
        }
        if (valid(l)) out[addr(l, k)] = acc + 2.0 * acc2;
    }
}

template <typename T>
__global__ void green_store(const double *a, int nx, int ny, int nz, double s, T *G, T *Gn) {
    const long total = static_cast<long>(nx + 1) * (ny + 1) * (nz + 1);
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const long kx = i % (nx + 1);
    const long row = i / (nx + 1);
    const T v = static_cast<T>(a[i] * s);
    if (kx < nx) G[row * nx + kx] = v;
    else Gn[row] = v;
}

template <typename T>
__global__ void green_load(const T *G, const T *Gn, int nx, int ny, int nz, T *dst) {
    const long total = static_cast<long>(nx + 1) * (ny + 1) * (nz + 1);
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const long kx = i % (nx + 1);
    const long row = i / (nx + 1);
    dst[i] = kx < nx ? G[row * nx + kx] : Gn[row];
}

static hipError_t axis_pass(const double *in, double *out, int A, int M, int B, const double *cos_tab,
                            hipStream_t stream) {
    // widest line tile whose lines plus cosine table fit in the 160 KB of LDS
    int tw = 16;
    while (tw > 1 && (static_cast<size_t>(M) * tw + 2 * (M - 1)) * sizeof(double) > 160 * 1024) tw /= 2;
    const size_t lds = (static_cast<size_t>(M) * tw + 2 * (M - 1)) * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(green_axis),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const long nblk = B > 1 ? static_cast<long>(A) * ((B + tw - 1) / tw) : (A + tw - 1) / tw;
    hipLaunchKernelGGL(green_axis, dim3(static_cast<unsigned>(nblk)), dim3(256), lds, stream, in, out, A, M, B, tw,
                       cos_tab);
    return hipGetLastError();
}

hipError_t green_spectrum(int nx, int ny, int nz, const double h[3], int prec, double *a, double *b,
                          const double *cos_x, const double *cos_y, const double *cos_z, void *G, void *Gn,
                          hipStream_t stream) {
    const long total = static_cast<long>(nx + 1) * (ny + 1) * (nz + 1);
    const unsigned nb = static_cast<unsigned>((total + 255) / 256);
    hipLaunchKernelGGL(green_fill, dim3(nb), dim3(256), 0, stream, nx, ny, nz, h[0], h[1], h[2], a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // x: [ (ny+1)(nz+1) ][ nx+1 ][ 1 ]
    if ((e = axis_pass(a, b, (ny + 1) * (nz + 1), nx + 1, 1, cos_x, stream)) != hipSuccess) return e;
    // y: [ nz+1 ][ ny+1 ][ nx+1 ]
    if ((e = axis_pass(b, a, nz + 1, ny + 1, nx + 1, cos_y, stream)) != hipSuccess) return e;
    // z: [ 1 ][ nz+1 ][ (nx+1)(ny+1) ]
    if ((e = axis_pass(a, b, 1, nz + 1, (nx + 1) * (ny + 1), cos_z, stream)) != hipSuccess) return e;
    const double s = 1.0 / (8.0 * nx * static_cast<double>(ny) * nz);
    if (prec == 0)
        hipLaunchKernelGGL(green_store<float>, dim3(nb), dim3(256), 0, stream, b, nx, ny, nz, s,
                           static_cast<float *>(G), static_cast<float *>(Gn));
    else
        hipLaunchKernelGGL(green_store<double>, dim3(nb), dim3(256), 0, stream, b, nx, ny, nz, s,
                           static_cast<double *>(G), static_cast<double *>(Gn));
    return hipGetLastError();
}

hipError_t green_export(int nx, int ny, int nz, int prec, const void *G, const void *Gn, void *dst,
                        hipStream_t stream) {
    const long total = static_cast<long>(nx + 1) * (ny + 1) * (nz + 1);
    const unsigned nb = static_cast<unsigned>((total + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(green_load<float>, dim3(nb), dim3(256), 0, stream, static_cast<const float *>(G),
                           static_cast<const float *>(Gn), nx, ny, nz, static_cast<float *>(dst));
    else
        hipLaunchKernelGGL(green_load<double>, dim3(nb), dim3(256), 0, stream, static_cast<const double *>(G),
                           static_cast<const double *>(Gn), nx, ny, nz, static_cast<double *>(dst));
    return hipGetLastError();
}

}  // namespace pspfft
