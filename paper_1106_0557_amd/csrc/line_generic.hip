// line_generic.hip -- the five passes for transform lengths outside the radix
// families of pass_kernels.h: any L = 2^a 3^b 5^c (odd parts beyond 1, 3, 5, 9,
// lines shorter than a family's element count, FP64 lines beyond the family
// limits).  Same passes, same workspace and spectrum layouts and the same
// unnormalised transforms as the family kernels (Sec. 2.1 mesh doubling, Sec.
// 2.2.2 sequence of 1D transforms), so one plan may mix family and generic axes.
//
// A workgroup of 256 threads owns `tile` whole lines (a power of two); each
// line gets 256 / tile threads, which walk its positions j0, j0 + tpl, ...  The
// lines are loaded into one of two LDS buffers; every stage (radices up to 27,
// Stockham autosort, decimation in time) reads one buffer and writes the other:
//   for each butterfly j < L/R of a line, k = j mod Ns:
//     x_r = in[j + r L/R] * exp(DIR 2 pi i r k / (Ns R)),  r < R
//     out[(j - k) R + k + r Ns] = DFT_R(x)[r]
// with Ns the product of the earlier radices; the result is in natural order.
// Column passes (y, z) keep element (line c, position p) at p*tile + c, so a
// wavefront's global accesses cover `tile` adjacent kx and its LDS accesses are
// consecutive; row passes (x) keep it at c*(L+1) + p.  Index arithmetic is
// shifts and adds: a thread's line is fixed, its positions advance by tpl, and
// k = j mod Ns advances by tpl mod Ns.
#include "fft_core.h"
#include "internal.h"

namespace pspfft {
namespace {

constexpr int kGenBlock = 256;
constexpr int kGenShift = 8;  // log2(kGenBlock)

template <bool ROW>
__device__ __forceinline__ int gidx(int c, int p, int tile, int L) {
    return ROW ? c * (L + 1) + p : p * tile + c;
}

// This thread's line of the tile and its first position; tpl threads per line.
struct GenMap {
    int c, j0, tpl;
};
template <bool ROW>
__device__ __forceinline__ GenMap gen_map(int tshift) {
    const int tid = static_cast<int>(threadIdx.x);
    GenMap m;
    m.tpl = kGenBlock >> tshift;
    if constexpr (ROW) {  // rows: consecutive lanes along a line
        m.c = tid >> (kGenShift - tshift);
        m.j0 = tid & (m.tpl - 1);
    } else {              // columns: consecutive lanes on adjacent lines
        m.c = tid & ((1 << tshift) - 1);
        m.j0 = tid >> tshift;
    }
    return m;
}

// One stage of radix R over the thread's butterflies of its line: src -> dst.
template <typename T, int R, int DIR, bool ROW>
__device__ void gen_stage(const cx<T> *src, cx<T> *dst, const GenMap &m, int tile, int L, int Ns,
                          const cx<T> *tw) {
    const int nb = L / R;  // butterflies per line
    int k = m.j0 % Ns;
    const int step = m.tpl % Ns;
    for (int j = m.j0; j < nb; j += m.tpl) {
        cx<T> x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = src[gidx<ROW>(m.c, j + r * nb, tile, L)];
        if (Ns > 1) {
            const cx<T> *t = tw + k * (R - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) x[r] = DIR > 0 ? cmulc(x[r], t[r - 1]) : cmul(x[r], t[r - 1]);
        }
        dft<R, DIR>(x);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[gidx<ROW>(m.c, base + r * Ns, tile, L)] = x[r];
        k += step;
        if (k >= Ns) k -= Ns;
    }
}

// Transform every line of the tile held in `a` (the other buffer `b` is
// scratch; `tw` the stage twiddle table, in LDS or global memory).  Returns the
// buffer that holds the result.  Opens with a barrier, so the caller's writes
// to `a` are visible, and ends with one.
template <typename T, int DIR, bool ROW>
__device__ cx<T> *gen_transform(cx<T> *a, cx<T> *b, const GenMap &m, int tile, const AxisPlan &ax,
                                const cx<T> *tw) {
    for (int s = 0; s < ax.nst; ++s) {
        __syncthreads();
        const cx<T> *t = tw + ax.twoff[s];
        const int L = ax.L, Ns = ax.Ns[s];
        switch (ax.R[s]) {
            case 2: gen_stage<T, 2, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 3: gen_stage<T, 3, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 4: gen_stage<T, 4, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 5: gen_stage<T, 5, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 6: gen_stage<T, 6, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 8: gen_stage<T, 8, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 9: gen_stage<T, 9, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 10: gen_stage<T, 10, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 12: gen_stage<T, 12, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 15: gen_stage<T, 15, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 16: gen_stage<T, 16, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 25: gen_stage<T, 25, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            case 27: gen_stage<T, 27, DIR, ROW>(a, b, m, tile, L, Ns, t); break;
            default: break;  // the host builds only these radices
        }
        cx<T> *tmp = a;
        a = b;
        b = tmp;
    }
    __syncthreads();
    return a;
}

// Column line g of a y pass (lines (z, kx), Nyquist lines z) or a z pass
// (lines (ky, kx), Nyquist lines ky): element p is base + p*step.  Position p
// of a y line is row w_row(z, p), linear in p; a z pass on this kernel has an
// untiled workspace (z tile 1), so its rows w_row(p, ky) are linear in p too.
template <typename T>
struct ColLineG {
    cx<T> *base;
    size_t step;
    __device__ __forceinline__ cx<T> &operator[](int p) const { return base[static_cast<size_t>(p) * step]; }
};
template <typename T, int MODE>
__device__ __forceinline__ ColLineG<T> col_line_g(const DevPlan &pl, cx<T> *W, cx<T> *Wn, bool nyq, long g) {
    const int nx = pl.nx, ny = pl.ny;
    if constexpr (MODE == Z_CONV) {
        if (nyq) return ColLineG<T>{Wn + g, static_cast<size_t>(2) * ny};
        const int ky = static_cast<int>(g / nx), kx = static_cast<int>(g - static_cast<long>(ky) * nx);
        return ColLineG<T>{W + w_row(0, ky, ny, nx, 1) + kx, static_cast<size_t>(2) * ny * nx};
    } else {
        if (nyq) return ColLineG<T>{Wn + static_cast<size_t>(g) * 2 * ny, 1};
        const int z = static_cast<int>(g / nx), kx = static_cast<int>(g - static_cast<long>(z) * nx);
        return ColLineG<T>{W + w_row(z, 0, ny, nx, pl.zb) + kx, static_cast<size_t>(pl.zb) * nx};
    }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kGenBlock) generic_kernel(const LaunchArgs args) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr bool ROW = (MODE == X_FWD || MODE == X_INV);
    constexpr int axis = ROW ? 0 : (MODE == Z_CONV ? 2 : 1);
    // XCD-aware order: workgroup b runs on XCD b mod 8; with the grid a whole
    // number of rounds of 64, tiles are dealt to the XCDs in chunks of 8
    // neighbours (chunk k to XCD k mod 8), so tiles that share 128-byte row
    // segments meet in one L2
    int bid = static_cast<int>(blockIdx.x);
    if ((gridDim.x & 63) == 0) {
        const int i = bid >> 3;
        bid = (((i >> 3) << 3) + (bid & 7)) * 8 + (i & 7);
    }
    if (bid >= args.nwg) return;
    int sgi = 0;
    while (sgi + 1 < args.nseg && bid >= args.seg[sgi + 1].wg_begin) ++sgi;
    const Segment &sg = args.seg[sgi];
    int local = bid - sg.wg_begin;
    const int member = local % sg.group;  // tile-major, as in the family kernels
    local /= sg.group;
    const ProbArg &pa = args.p[sg.first + member];
    const DevPlan &pl = *pa.plan;
    const AxisPlan &ax = pl.ax[axis];
    const int nx = pl.nx, ny = pl.ny, nz = pl.nz;
    const int L = ax.L;
    const int tile = args.gtile;
    const int tshift = __builtin_ctz(static_cast<unsigned>(tile));
    cx<T> *A = reinterpret_cast<cx<T> *>(smem);
    cx<T> *B = A + static_cast<size_t>(tile) * (L + 1);
    // stage twiddles: in LDS after the two buffers of the launch's longest line
    // when the host found room (args.gtw), else read from the plan's table
    const cx<T> *tw = static_cast<const cx<T> *>(ax.tw);
    if (args.gtw) {
        cx<T> *twl = A + static_cast<size_t>(2) * tile * (args.glmax + 1);
        for (int i = static_cast<int>(threadIdx.x); i < ax.ntw; i += kGenBlock) twl[i] = tw[i];
        tw = twl;  // published by the first stage's barrier
    }
    cx<T> *W = static_cast<cx<T> *>(pa.W);
    cx<T> *Wn = static_cast<cx<T> *>(pa.Wn);
    const bool nyq = local >= sg.wg_main;
    if (nyq) local -= sg.wg_main;
    const GenMap m = gen_map<ROW>(tshift);
    const long g = static_cast<long>(local) * tile + m.c;  // this thread's line
    const cx<T> zero = {T(0), T(0)};

    if constexpr (MODE == X_FWD) {
        // rows r = z*ny + y of S, zero-padded to 2nx, packed u[j] = s[2j] + i s[2j+1] (L = nx)
        const bool active = g < static_cast<long>(ny) * nz;
        const T *row = static_cast<const T *>(pa.S) + static_cast<size_t>(active ? g : 0) * nx;
        for (int j = m.j0; j < L; j += m.tpl) {
            cx<T> v = zero;
            if (active) {
                if (2 * j < nx) v.x = row[2 * j];
                if (2 * j + 1 < nx) v.y = row[2 * j + 1];
            }
            A[gidx<true>(m.c, j, tile, L)] = v;
        }
        const cx<T> *U = gen_transform<T, -1, true>(A, B, m, tile, ax, tw);
        if (active) {
            // split step: X[k] = (U[k] + U*[n-k])/2 - (i/2) exp(-i pi k/n) (U[k] - U*[n-k]), k <= n
            const cx<T> *post = static_cast<const cx<T> *>(ax.post);
            const int z = static_cast<int>(g / ny), y = static_cast<int>(g - static_cast<long>(z) * ny);
            cx<T> *wrow = W + w_row(z, y, ny, nx, pl.zb);
            for (int k = m.j0; k <= L; k += m.tpl) {
                const cx<T> u = U[gidx<true>(m.c, k == L ? 0 : k, tile, L)];
                const cx<T> w = U[gidx<true>(m.c, k == 0 ? 0 : L - k, tile, L)];
                const cx<T> a = {static_cast<T>(0.5) * (u.x + w.x), static_cast<T>(0.5) * (u.y - w.y)};
                const cx<T> b = {static_cast<T>(0.5) * (u.x - w.x), static_cast<T>(0.5) * (u.y + w.y)};
                const cx<T> e = k < L ? post[k] : cx<T>{T(-1), T(0)};
                const cx<T> eb = cmul(e, b);
                const cx<T> X = {a.x + eb.y, a.y - eb.x};  // a - i e b
                if (k < nx) wrow[k] = X;
                else Wn[static_cast<size_t>(z) * 2 * ny + y] = X;
            }
        }
    } else if constexpr (MODE == X_INV) {
        // X[k], k <= n, of rows y < ny; Hermitian extension through the inverse split step
        const bool active = g < static_cast<long>(ny) * nz;
        const int z = active ? static_cast<int>(g / ny) : 0;
        const int y = active ? static_cast<int>(g - static_cast<long>(z) * ny) : 0;
        const cx<T> *wrow = W + w_row(z, y, ny, nx, pl.zb);
        for (int k = m.j0; k <= L; k += m.tpl) {
            cx<T> v = zero;
            if (active) v = k < nx ? wrow[k] : Wn[static_cast<size_t>(z) * 2 * ny + y];
            B[gidx<true>(m.c, k, tile, L)] = v;  // L + 1 slots per row
        }
        __syncthreads();
        // U[k] = (X[k] + X*[n-k]) + i exp(+i pi k/n) (X[k] - X*[n-k]), k < n
        const cx<T> *post = static_cast<const cx<T> *>(ax.post);
        for (int k = m.j0; k < L; k += m.tpl) {
            const cx<T> xk = B[gidx<true>(m.c, k, tile, L)];
            const cx<T> xm = B[gidx<true>(m.c, L - k, tile, L)];
            const cx<T> e = {xk.x + xm.x, xk.y - xm.y};
            const cx<T> o = cmulc(cx<T>{xk.x - xm.x, xk.y + xm.y}, post[k]);  // times exp(+i pi k/n)
            A[gidx<true>(m.c, k, tile, L)] = cx<T>{e.x - o.y, e.y + o.x};   // e + i o
        }
        const cx<T> *u = gen_transform<T, +1, true>(A, B, m, tile, ax, tw);
        if (active) {
            T *Phi = static_cast<T *>(pa.Phi) + static_cast<size_t>(g) * nx;
            for (int x = m.j0; x < nx; x += m.tpl) {
                const cx<T> v = u[gidx<true>(m.c, x >> 1, tile, L)];
                Phi[x] = (x & 1) ? v.y : v.x;
            }
        }
    } else {
        // column lines: y passes over (z, kx), z pass over (ky, kx); Nyquist lines kx = nx
        long nlines;
        int nin, nout;  // positions read (the rest is zero padding) and written
        if constexpr (MODE == Z_CONV) {
            nlines = nyq ? 2L * ny : 2L * ny * nx;
            nin = nz;
            nout = nz;
        } else {
            nlines = nyq ? static_cast<long>(nz) : static_cast<long>(nz) * nx;
            nin = MODE == Y_FWD ? ny : L;
            nout = MODE == Y_FWD ? L : ny;
        }
        const bool active = g < nlines;
        const ColLineG<T> line = col_line_g<T, MODE>(pl, W, Wn, nyq, active ? g : 0);
        for (int p = m.j0; p < L; p += m.tpl) {
            cx<T> v = zero;
            if (active && p < nin) v = line[p];
            A[gidx<false>(m.c, p, tile, L)] = v;
        }
        cx<T> *res;
        if constexpr (MODE == Z_CONV) {
            res = gen_transform<T, -1, false>(A, B, m, tile, ax, tw);
            // multiply by the spectrum, even in ky and kz: octant index min(k, 2n - k)
            if (active) {
                const T *G = static_cast<const T *>(pl.G);
                const T *Gn = static_cast<const T *>(pl.Gn);
                const int ky = nyq ? static_cast<int>(g) : static_cast<int>(g / nx);
                const int kx = nyq ? nx : static_cast<int>(g - static_cast<long>(ky) * nx);
                const int kyo = ky <= ny ? ky : 2 * ny - ky;
                // plans with generic z lines keep the spectrum kz-fastest: octant value
                // (kyo, kx, kzo) at (kyo*nx + kx)*(nz + 1) + kzo, Nyquist column kyo*(nz + 1) + kzo,
                // so the lanes of a line read consecutive values
                const T *gl = nyq ? Gn + static_cast<size_t>(kyo) * (nz + 1)
                                  : G + (static_cast<size_t>(kyo) * nx + kx) * (nz + 1);
                for (int kz = m.j0; kz < L; kz += m.tpl) {
                    const int kzo = kz <= nz ? kz : L - kz;
                    const T gv = gl[kzo];
                    cx<T> &e = res[gidx<false>(m.c, kz, tile, L)];
                    e = cx<T>{e.x * gv, e.y * gv};
                }
            }
            res = gen_transform<T, +1, false>(res, res == A ? B : A, m, tile, ax, tw);
        } else {
            res = gen_transform<T, MODE == Y_FWD ? -1 : +1, false>(A, B, m, tile, ax, tw);
        }
        if (active) {
            for (int p = m.j0; p < nout; p += m.tpl) line[p] = res[gidx<false>(m.c, p, tile, L)];
        }
    }
}

template <typename T, int MODE>
hipError_t launch_gen(const LaunchArgs &args, int grid, size_t lds, hipStream_t stream) {
    static bool attr_set = false;
    auto fn = generic_kernel<T, MODE>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kGenBlock), lds, stream, args);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gen_mode(int mode, const LaunchArgs &args, int grid, size_t lds, hipStream_t stream) {
    switch (mode) {
        case X_FWD: return launch_gen<T, X_FWD>(args, grid, lds, stream);
        case Y_FWD: return launch_gen<T, Y_FWD>(args, grid, lds, stream);
        case Z_CONV: return launch_gen<T, Z_CONV>(args, grid, lds, stream);
        case Y_INV: return launch_gen<T, Y_INV>(args, grid, lds, stream);
        case X_INV: return launch_gen<T, X_INV>(args, grid, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_generic(int mode, int prec, const LaunchArgs &args, int grid, size_t lds, hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    return prec == 0 ? launch_gen_mode<float>(mode, args, grid, lds, stream)
                     : launch_gen_mode<double>(mode, args, grid, lds, stream);
}

}  // namespace pspfft
