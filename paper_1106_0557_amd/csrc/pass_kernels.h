// pass_kernels.h -- the five streaming passes of one mesh-doubling solve
// (Budiardja & Cardall, arXiv:1106.0557, Sec. 2.1 and 2.2.2) as gfx950 kernels.
//
//   X_FWD  : rows of S, zero-padded to 2nx, transformed along x (packed real form)
//   Y_FWD  : columns along y; the input half y >= ny is zero and never read
//   Z_CONV : columns along z: forward transform (input half zero), multiply by the
//            Green's-function spectrum, inverse transform, keep z < nz (Sec. 2.1,
//            convolution theorem; Sec. 2.2.2, the multiply happens in z pillars)
//   Y_INV  : inverse along y, keep y < ny
//   X_INV  : inverse along x with the Hermitian extension, keep x < nx -> Phi
// The normalisation 1/((2nx)(2ny)(2nz)) is folded into the spectrum.
//
// Line engine.  A line of length L is owned by NB = L/E threads of a workgroup;
// thread t holds positions t + NB*m (m < E) in registers.  Stages (Stockham,
// decimation in time) have radix E first, then M (the power-of-two part of E) in
// the middle, then K last; every radix divides E, so each thread applies E/R
// butterflies per stage.  Stage 0 reads the registers the caller loaded from
// global memory and scatters to LDS; middle stages go LDS -> LDS; the last stage
// gathers from LDS and leaves its outputs in the thread's own positions, in
// registers.  E and K are template parameters, so no line data is carried in
// registers across a runtime branch or loop back-edge.  The zero half of an input
// and the discarded half of an output are registers m >= E/2, known at compile
// time, so their butterfly arithmetic is removed by the compiler.
#pragma once

#include "fft_core.h"
#include "internal.h"

namespace pspfft {

// Global-address-space view of a pointer that came from device memory (the
// compiler cannot infer it), so its loads are global rather than flat ones.
template <typename U>
using gbl = __attribute__((address_space(1))) U;
template <typename U>
__device__ __forceinline__ const gbl<U> *as_global(const U *p) {
    return (const gbl<U> *)p;
}
// Nontemporal accesses of one complex value in global memory (streamed data
// that should not displace what later accesses of the launch reuse).
template <typename T>
__device__ __forceinline__ void st_nt(cx<T> *p, cx<T> v) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(__builtin_bit_cast(v2, v), (__attribute__((address_space(1))) v2 *)(p));
}
template <typename T>
__device__ __forceinline__ cx<T> ld_nt(const cx<T> *p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(cx<T>, __builtin_nontemporal_load((const __attribute__((address_space(1))) v2 *)(p)));
}

// Stage twiddle w of a table in LDS (a generic pointer) or in global memory.
template <typename T>
__device__ __forceinline__ cx<T> tw_at(const cx<T> *p, int i) {
    return p[i];
}
template <typename T>
__device__ __forceinline__ cx<T> tw_at(const gbl<cx<T>> *p, int i) {
    return cx<T>{p[i].x, p[i].y};
}

// CNB, CLDSW: threads per line and LDS stride when known at compile time (a
// two-stage line, L = E*K and CNB = K; three stages with radices E, M, K,
// L = E*M*K and CNB = M*K; or four, E, M, M, K, L = E*M*M*K and CNB = M*M*K),
// else 0.
template <typename T, int E, int DIR, bool ROW, int CNB = 0, int CLDSW = 0>
struct LineFFT {
    static constexpr int M = E & -E;  // radix of the middle stages

    // LDS layout: column passes keep (line c, position P) at P*ldsw + c with
    // ldsw = col_stride(); row passes at c*ldsw + P + P/16 with ldsw = row_stride().
    static __device__ __forceinline__ void gather(cx<T> *v, const cx<T> *lds, int ldsw_, int c, int t, int NB_) {
        const int NB = CNB ? CNB : NB_;
        const int ldsw = CLDSW ? CLDSW : ldsw_;
        if constexpr (ROW && CNB != 0 && CNB % 16 == 0) {
            // P = t + NB*m with NB a multiple of 16: P + P/16 = t + t/16 + m*(NB + NB/16)
            const cx<T> *p0 = lds + c * ldsw + t + (t >> 4);
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = p0[m * (CNB + CNB / 16)];
        } else if constexpr (ROW) {
            const cx<T> *row = lds + c * ldsw;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int P = t + NB * m;
                v[m] = row[P + (P >> 4)];
            }
        } else {
            const cx<T> *col = lds + t * ldsw + c;
            const int step = NB * ldsw;
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = col[m * step];
        }
    }

    // E/R radix-R butterflies on the thread's registers.  Stage parameters:
    // Ns = product of the earlier radices, mg its division magic, tw the stage's
    // twiddle table.  TW: multiply by twiddles (every stage but the first).
    // TO_LDS: scatter the outputs to their Stockham positions in LDS; otherwise
    // (last stage) they land in the thread's own positions, in registers.
    template <int R, bool TW, bool TO_LDS, int CNS = 0, typename TP = const cx<T> *>
    static __device__ __forceinline__ void stage(cx<T> *v, int Ns_, uint32_t mg, TP tw, cx<T> *lds,
                                                 int ldsw_, int c, int t, int NB_) {
        constexpr int NBF = E / R;
        const int NB = CNB ? CNB : NB_;
        const int ldsw = CLDSW ? CLDSW : ldsw_;
        const int Ns = CNS ? CNS : Ns_;
        sfor<0, NBF>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const int b = t + NB * i;
            int q = b, k = 0;
            if constexpr (TW) {
                if constexpr (CNS != 0) q = b / CNS;
                else q = static_cast<int>(__umulhi(static_cast<uint32_t>(b), mg));
                k = b - q * Ns;
            }
            cx<T> x[R];
            sfor<0, R>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                x[r] = v[i + r * NBF];
            });
            if constexpr (TW) {
                const TP twk = tw + k * (R - 1);
                sfor<1, R>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    const cx<T> w = tw_at(twk, r - 1);
                    if constexpr (DIR > 0) x[r] = cmulc(x[r], w);
                    else x[r] = cmul(x[r], w);
                });
            }
            dft<R, DIR>(x);
            if constexpr (TO_LDS) {
                const int base = q * Ns * R + k;  // output r goes to position base + r*Ns
                if constexpr (ROW && ((CNS != 0 && CNS % 16 == 0) || (!TW && 16 % R == 0))) {
                    // Ns a multiple of 16: P + P/16 = base + base/16 + r*(Ns + Ns/16); first
                    // stage (Ns = 1, base = b*R) with R dividing 16: base + base/16 + r
                    constexpr int RS = TW ? CNS + CNS / 16 : 1;
                    cx<T> *p0 = lds + c * ldsw + base + (base >> 4);
                    sfor<0, R>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        p0[r * RS] = x[r];
                    });
                } else if constexpr (ROW) {
                    cx<T> *row = lds + c * ldsw;
                    sfor<0, R>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        const int P = base + r * Ns;
                        row[P + (P >> 4)] = x[r];
                    });
                } else {
                    cx<T> *col = lds + base * ldsw + c;
                    const int step = Ns * ldsw;
                    sfor<0, R>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        col[r * step] = x[r];
                    });
                }
            } else {
                sfor<0, R>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    v[i + r * NBF] = x[r];
                });
            }
        });
    }

    // Transform the line whose positions t + NB*m the thread holds in v[m].
    // K = radix of the last stage (1: the whole line is one radix-E stage).
    // twl: stage twiddle tables in LDS, published by the first barrier (or in
    // global memory: a global-address-space pointer).
    // LEAD: open with a barrier so that earlier readers of the line's LDS
    // region are done; a caller that has just passed a barrier can skip it.
    // WAVE: every line lies within one wavefront (its LDS region too), so the
    // exchanges need only the wavefront's own in-order LDS accesses; the
    // barriers become compiler ordering points.
    template <bool WAVE>
    static __device__ __forceinline__ void sync() {
        if constexpr (WAVE) __builtin_amdgcn_wave_barrier();
        else __syncthreads();
    }

    template <int K, bool LEAD = true, bool WAVE = false, typename TP = const cx<T> *>
    static __device__ __forceinline__ void run(cx<T> *v, const AxisPlan &ax, cx<T> *lds, int ldsw,
                                               TP twl, int c, int t) {
        const int NB = CNB ? CNB : ax.NB;
        if constexpr (K == 1) {
            stage<E, false, false>(v, 1, 0u, twl, lds, ldsw, c, t, NB);
        } else if constexpr (CNB == K) {
            // two stages, radix E then K: the second has Ns = E and its twiddles
            // follow the E - 1 entries of the first
            if constexpr (LEAD) sync<WAVE>();  // earlier readers of LDS are done
            stage<E, false, true>(v, 1, 0u, twl, lds, ldsw, c, t, NB);
            sync<WAVE>();
            gather(v, lds, ldsw, c, t, NB);
            stage<K, true, false, E>(v, E, 0u, twl + (E - 1), lds, ldsw, c, t, NB);
        } else if constexpr (CNB != 0 && CNB == M * M * K) {
            // four stages, radices E, M, M, K: Ns = 1, E, E*M, E*M*M; the twiddle
            // tables follow one another (E - 1, E*(M - 1) and E*M*(M - 1) entries)
            if constexpr (LEAD) sync<WAVE>();
            stage<E, false, true>(v, 1, 0u, twl, lds, ldsw, c, t, NB);
            sync<WAVE>();
            gather(v, lds, ldsw, c, t, NB);
            sync<WAVE>();
            stage<M, true, true, E>(v, E, 0u, twl + (E - 1), lds, ldsw, c, t, NB);
            sync<WAVE>();
            gather(v, lds, ldsw, c, t, NB);
            sync<WAVE>();
            stage<M, true, true, E * M>(v, E * M, 0u, twl + (E - 1) + E * (M - 1), lds, ldsw, c, t, NB);
            sync<WAVE>();
            gather(v, lds, ldsw, c, t, NB);
            stage<K, true, false, E * M * M>(v, E * M * M, 0u, twl + (E - 1) + E * (M - 1) + E * M * (M - 1), lds,
                                             ldsw, c, t, NB);
        } else if constexpr (CNB != 0) {
            // three stages, radices E, M, K (CNB = M*K): Ns = 1, E, E*M; the
            // twiddle tables follow one another (E - 1 and E*(M - 1) entries)
            static_assert(CNB == M * K, "compile-time lines have two, three or four stages");
            if constexpr (LEAD) sync<WAVE>();
            stage<E, false, true>(v, 1, 0u, twl, lds, ldsw, c, t, NB);
            sync<WAVE>();
            gather(v, lds, ldsw, c, t, NB);
            sync<WAVE>();
            stage<M, true, true, E>(v, E, 0u, twl + (E - 1), lds, ldsw, c, t, NB);
            sync<WAVE>();
            gather(v, lds, ldsw, c, t, NB);
            stage<K, true, false, E * M>(v, E * M, 0u, twl + (E - 1) + E * (M - 1), lds, ldsw, c, t, NB);
        } else {
            if constexpr (LEAD) sync<WAVE>();  // earlier readers of LDS are done
            stage<E, false, true>(v, 1, 0u, twl, lds, ldsw, c, t, NB);
            const int last = ax.nst - 1;
            for (int s = 1; s < last; ++s) {
                sync<WAVE>();
                gather(v, lds, ldsw, c, t, NB);
                sync<WAVE>();
                stage<M, true, true>(v, ax.Ns[s], ax.magic[s], twl + ax.twoff[s], lds, ldsw, c, t, NB);
            }
            sync<WAVE>();
            gather(v, lds, ldsw, c, t, NB);
            stage<K, true, false>(v, ax.Ns[last], ax.magic[last], twl + ax.twoff[last], lds, ldsw, c, t, NB);
        }
    }
};

// Value of another lane of the wavefront (byte address src_lane*4), through the
// LDS crossbar without LDS storage or a barrier.
__device__ __forceinline__ float lane_read(int addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_read(int addr, double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, static_cast<int>(b));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, static_cast<int>(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Mirror partners of a packed real transform.  The NB (a power of two that
// divides 64) threads of a row are consecutive lanes; thread t (lane `lane` of
// the wavefront) holds positions k = t + NB*m of a length n = E*NB line.  p[m]
// receives the value at position (n - k) mod n, which thread (NB - t) mod NB
// holds in register E - 1 - m (t > 0) and thread 0 holds in its own register
// (E - m) mod E.
template <typename T, int E, int NB>
__device__ __forceinline__ void mirror_partners(const cx<T> *v, cx<T> *p, int t, int lane) {
    if constexpr (NB == 1) {
#pragma unroll
        for (int m = 0; m < E; ++m) p[m] = v[(E - m) % E];
    } else {
        const int addr = (lane - t + ((NB - t) & (NB - 1))) << 2;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const cx<T> d = t == 0 ? v[(E - m) % E] : v[E - 1 - m];  // what this lane sends
            p[m] = cx<T>{lane_read(addr, d.x), lane_read(addr, d.y)};
        }
    }
}

template <typename T>
__device__ __forceinline__ void copy_to_lds(cx<T> *dst, const void *src, int count) {
    const cx<T> *s = static_cast<const cx<T> *>(src);
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = s[i];
}


// Element m of a line: base + lane + m*step bytes.  OFF32 (set by the host when
// every array of the launch is below 4 GB): the offset lane + m*step is
// computed in 32 bits and added to the workgroup-uniform base, so each access
// is a scalar base plus one 32-bit vector offset.
template <typename T, bool OFF32>
struct LinePtr {
    char *base;
    size_t lane;
    size_t step;
    __device__ __forceinline__ cx<T> &operator[](int m) const {
        if constexpr (OFF32)
            return *reinterpret_cast<cx<T> *>(
                base + (static_cast<uint32_t>(lane) + static_cast<uint32_t>(m) * static_cast<uint32_t>(step)));
        else
            return *reinterpret_cast<cx<T> *>(base + lane + static_cast<size_t>(m) * step);
    }
};
template <typename T, bool OFF32>
__device__ __forceinline__ LinePtr<T, OFF32> line_ptr(const void *base, size_t lane_elems, size_t step_elems,
                                                      size_t esz) {
    return LinePtr<T, OFF32>{const_cast<char *>(static_cast<const char *>(base)), lane_elems * esz, step_elems * esz};
}

// Element m of a line in an array of 4 GB or more whose lane offsets stay below
// the position stride (z lines: a lane's offset within its NB-position block):
// a workgroup-uniform 64-bit base per position block, base + m*step, plus one
// 32-bit lane offset.
template <typename T>
struct LinePtrW {
    char *base;
    size_t lane;
    size_t step;
    __device__ __forceinline__ char *block(int m) const { return base + static_cast<size_t>(m) * step; }
    __device__ __forceinline__ cx<T> &operator[](int m) const {
        return *reinterpret_cast<cx<T> *>(block(m) + static_cast<uint32_t>(lane));
    }
};

// fix_stages(FIX) (2, 3 or 4): every problem of the launch has lines of that
// many stages with radices E, (M, (M,)) K and the workgroup holds pass_tile()
// lines, so the geometry is compile-time.  fix_off32(FIX): every array is below
// 4 GB, so addresses use 32-bit lane offsets; otherwise (FIX & kFixWide) 64-bit
// addresses.  FIX = 0: geometry from the plan at run time, 64-bit addresses.
// NT (z lines of a streaming launch): the line is loaded and stored with
// nontemporal accesses, so that it does not displace the spectrum, which the
// launch's problems share.
template <typename T, int E, int K, int MODE, int FIX, bool NT = false>
__global__ void __launch_bounds__((max_block_for(sizeof(T) == 4 ? 0 : 1, E))) pass_kernel(const LaunchArgs args) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem);
    constexpr bool ROW = (MODE == X_FWD || MODE == X_INV);
    constexpr int H = E / 2;  // registers m < H hold the first half of the line
    constexpr int CSZ = static_cast<int>(sizeof(cx<T>));
    constexpr int ST = fix_stages(FIX);  // compile-time stages (0: run-time geometry)
    constexpr bool OFF32 = fix_off32(FIX);
    constexpr int CNB = fix_nb(FIX, E, K);
    constexpr int FTILE = pass_tile(sizeof(T) == 4 ? 0 : 1, MODE, E, CNB);
    constexpr int CL = E * CNB;  // line length when compile-time
    constexpr int PREC = sizeof(T) == 4 ? 0 : 1;
    constexpr int CLDSW = ST ? (ROW ? row_stride(CL, CNB, CSZ) : col_ldsw(PREC, MODE, E, CNB)) : 0;
    using FFT_F = LineFFT<T, E, -1, ROW, CNB, CLDSW>;
    using FFT_I = LineFFT<T, E, +1, ROW, CNB, CLDSW>;
    // compile-time rows of at most 64 threads are consecutive lanes of one
    // wavefront, as is their LDS row: their exchanges need no workgroup barrier,
    // and the partners of the split step come from the mirror lane
    constexpr bool RW = ROW && ST != 0 && CNB <= 64;

    // XCD-aware order: hardware hands consecutive workgroups to the 8 XCDs in
    // turn; renumber so that each XCD works through a contiguous range of the
    // launch (neighbouring tiles, and the same tile of batched problems that
    // share a spectrum, then meet in one L2).
    const int nwg = static_cast<int>(gridDim.x);
    const int bx = static_cast<int>(blockIdx.x);
    int bid = bx;
    if (args.xcd_remap == 1) {         // each XCD takes one contiguous eighth of the launch
        const int per = nwg >> 3;      // the grid is a multiple of 8 when remapping
        bid = (bx & 7) * per + (bx >> 3);
    } else if (args.xcd_remap == 2) {  // within each block of 64, each XCD takes 8 in a row
        bid = (bx & ~63) + ((bx & 7) << 3) + ((bx >> 3) & 7);
    }
    if (bid >= args.nwg) return;  // padding of the grid to a multiple of 8
    int sgi = 0;
    while (sgi + 1 < args.nseg && bid >= args.seg[sgi + 1].wg_begin) ++sgi;
    const Segment &sg = args.seg[sgi];
    int local = bid - sg.wg_begin;
    const int member = local % sg.group;  // segments are tiled tile-major
    local /= sg.group;
    const ProbArg &pa = args.p[sg.first + member];
    const DevPlan &pl = *pa.plan;
    constexpr int axis = ROW ? 0 : (MODE == Z_CONV ? 2 : 1);
    const AxisPlan &ax = pl.ax[axis];
    const int nx = pl.nx, ny = pl.ny, nz = pl.nz;
    const int NB = ST ? CNB : ax.NB;
    const int L = ST ? CL : ax.L;
    const int block = ST ? FTILE * CNB : static_cast<int>(blockDim.x);
    const int tile = ST ? FTILE : block / NB;  // lines per workgroup (power of two)
    const int tid = threadIdx.x;
    int c, t;
    if constexpr (ROW) {  // rows are contiguous in memory: consecutive lanes walk along a row
        t = tid & (NB - 1);
        c = tid >> __builtin_ctz(NB);
    } else {              // columns: consecutive lanes take adjacent lines (adjacent kx)
        c = tid & (tile - 1);
        t = tid >> __builtin_ctz(tile);
    }
    const int ldsw = ST ? CLDSW : (ROW ? row_stride(L, NB, CSZ) : col_stride(L, tile, CSZ));
    // GT: compile-time rows whose stage twiddles and split factors stay in
    // global memory (row_tables_global), or column y lines whose twiddles do
    // (col_tables_global, positions packed); else the tables follow the data in LDS
    constexpr bool GT = ST != 0 && (ROW ? row_tables_global(PREC, E, CNB) : col_tables_global(PREC, MODE, E, CNB));
    cx<T> *twd = lds + (ST ? (ROW ? data_elems(true, CL, CNB, FTILE * CNB, CSZ) : CL * CLDSW)
                           : data_elems(ROW, L, NB, block, CSZ));
    if constexpr (!GT) copy_to_lds<T>(twd, ax.tw, ax.ntw);
    const auto twl = [&]() __attribute__((always_inline)) {
        if constexpr (GT) return as_global(static_cast<const cx<T> *>(ax.tw));
        else return static_cast<const cx<T> *>(twd);
    }();

    const bool nyq = local >= sg.wg_main;
    if (nyq) local -= sg.wg_main;
    const int g = local * tile + c;  // line index within its set

    cx<T> v[E];
    cx<T> *W = static_cast<cx<T> *>(pa.W);
    cx<T> *Wn = static_cast<cx<T> *>(pa.Wn);

    if constexpr (ROW) {
        // Rows (y, z), y < ny, z < nz; row r = z*ny + y.  Packed real transform of
        // length n: u[j] = s[2j] + i s[2j+1], zero for j >= n/2 (the padding).
        // exp(-i pi k / n), k < n
        const auto post = [&]() __attribute__((always_inline)) {
            if constexpr (GT) {
                return as_global(static_cast<const cx<T> *>(ax.post));
            } else {
                cx<T> *p = twd + ax.ntw;
                copy_to_lds<T>(p, ax.post, L);
                return static_cast<const cx<T> *>(p);
            }
        }();
        const int nrows = ny * nz;
        const bool active = g < nrows;
        const int z = active ? g / ny : 0;
        const int y = g - z * ny;
        const size_t wrow = w_row(z, y, ny, nx, pl.zb);  // row start in W (elements)
        cx<T> *wnyq = Wn + static_cast<size_t>(z) * 2 * ny + y;
        // thread t's positions t + NB*m of row g of S / Phi (pairs of reals) and of W
        const auto fld = line_ptr<T, OFF32>(MODE == X_FWD ? pa.S : pa.Phi,
                                          static_cast<size_t>(active ? g : 0) * nx / 2 + t, NB, CSZ);
        const auto wl = line_ptr<T, OFF32>(W, wrow + t, NB, CSZ);
        if constexpr (MODE == X_FWD) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m < H && active) v[m] = fld[m];
                else v[m] = cx<T>{T(0), T(0)};
            }
            if constexpr (RW) {
                __syncthreads();  // twiddles visible
                FFT_F::template run<K, false, true>(v, ax, lds, ldsw, twl, c, t);
            } else {
                FFT_F::template run<K>(v, ax, lds, ldsw, twl, c, t);
            }
            // split: X[k] = (U[k] + U*[n-k])/2 - (i/2) exp(-i pi k/n) (U[k] - U*[n-k]).
            // Partners U[n-k]: from the mirror lane of the row with compile-time
            // geometry, else through the row in LDS.
            cx<T> wp[E];
            if constexpr (RW) {
                mirror_partners<T, E, CNB>(v, wp, t, tid & 63);
            } else {
                __syncthreads();
                cx<T> *row = lds + c * ldsw;
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int P = t + NB * m;
                    row[P + (P >> 4)] = v[m];
                }
                __syncthreads();
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int k = t + NB * m;
                    const int kp = k == 0 ? 0 : L - k;
                    wp[m] = row[kp + (kp >> 4)];
                }
            }
            if (active) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int k = t + NB * m;
                    const cx<T> u = v[m];
                    const cx<T> w = wp[m];
                    const cx<T> a = {static_cast<T>(0.5) * (u.x + w.x), static_cast<T>(0.5) * (u.y - w.y)};
                    const cx<T> b = {static_cast<T>(0.5) * (u.x - w.x), static_cast<T>(0.5) * (u.y + w.y)};
                    const cx<T> eb = cmul(tw_at(post, k), b);
                    wl[m] = cx<T>{a.x + eb.y, a.y - eb.x};  // a - i e b
                    if (k == 0) *wnyq = cx<T>{u.x - u.y, T(0)};
                }
            }
        } else {
            // U[k] = (X[k] + X*[n-k]) + i exp(+i pi k/n) (X[k] - X*[n-k]), k < n.
            // Each thread loads its own X[k]; the partners come through LDS.
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (active) v[m] = wl[m];
                else v[m] = cx<T>{T(0), T(0)};
            }
            cx<T> xn = {T(0), T(0)};
            if (active) xn = *wnyq;
            // partners X[n-k] (X[n] for k = 0): mirror lane, or through the row in LDS
            cx<T> wp[E];
            if constexpr (RW) {
                mirror_partners<T, E, CNB>(v, wp, t, tid & 63);
                __syncthreads();  // post table and twiddles visible
            } else {
                cx<T> *row = lds + c * ldsw;
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int P = t + NB * m;
                    row[P + (P >> 4)] = v[m];
                }
                __syncthreads();  // row values, post table and twiddles visible
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int k = t + NB * m;
                    const int kp = k == 0 ? 0 : L - k;  // k = 0 takes X[n] below
                    wp[m] = row[kp + (kp >> 4)];
                }
            }
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int k = t + NB * m;
                const cx<T> a = v[m];
                const cx<T> b = k == 0 ? xn : wp[m];
                const cx<T> sm = {a.x + b.x, a.y - b.y};
                const cx<T> df = {a.x - b.x, a.y + b.y};
                const cx<T> ed = cmulc(df, tw_at(post, k));
                v[m] = cx<T>{sm.x - ed.y, sm.y + ed.x};
            }
            // with the mirror lanes nothing of the row is in LDS yet: no leading barrier
            FFT_I::template run<K, !RW, RW>(v, ax, lds, ldsw, twl, c, t);
            if (active) {
#pragma unroll
                for (int m = 0; m < H; ++m) fld[m] = v[m];
            }
        }
    } else {
        // Column passes: line g starts at element `base` of `arr`, elements `es` apart.
        const cx<T> *arr;
        size_t base, es;
        bool active;
        int ky = 0, kx = 0;
        if constexpr (MODE == Z_CONV) {
            // Rows of the plane are visited in the order 0, 1, 2ny-1, 2, 2ny-2, ...,
            // ny, so that ky and its mirror 2ny - ky (same spectrum values) are
            // handled by neighbouring workgroups.
            if (!nyq) {
                active = g < 2 * ny * nx;
                const int vrow = active ? g / nx : 0;
                kx = g - vrow * nx;
                ky = vrow == 0 ? 0 : (vrow == 2 * ny - 1 ? ny : ((vrow & 1) ? (vrow + 1) >> 1 : 2 * ny - (vrow >> 1)));
                arr = W;
                base = static_cast<size_t>(ky) * pl.zb * nx + kx;
                es = static_cast<size_t>(2) * ny * nx;  // per z tile of the threads' positions, see below
            } else {
                active = g < 2 * ny;
                ky = g;
                kx = nx;
                arr = Wn;
                base = static_cast<size_t>(g);
                es = static_cast<size_t>(2) * ny;
            }
        } else {
            if (!nyq) {
                active = g < nz * nx;
                const int z = active ? g / nx : 0;
                kx = g - z * nx;
                arr = W;
                base = w_row(z, 0, ny, nx, pl.zb) + kx;
                es = static_cast<size_t>(pl.zb) * nx;
            } else {
                active = g < nz;
                arr = Wn;
                base = static_cast<size_t>(active ? g : 0) * 2 * ny;
                es = 1;
            }
        }
        // this thread's position t; position t + NB*m is m*NB*es elements further.
        // z lines of the main part: z = t + NB*m sits in tile z/zb at row z%zb,
        // and zb divides NB, so the thread's offset is fixed and each m moves
        // NB/zb tiles of 2ny*zb*nx elements.  An inactive line (past the end of
        // a partial tile) reads in-bounds dummies from the start of the array and
        // stores nothing.
        size_t lane_off = base + t * es;
        if (MODE == Z_CONV && !nyq) {
            const int zb = pl.zb;
            const int sh = __builtin_ctz(static_cast<unsigned>(zb));
            lane_off = base + (static_cast<size_t>(t >> sh) * 2 * ny * zb + (t & (zb - 1))) * nx;
        }
        const auto lane = line_ptr<T, OFF32>(arr, active ? lane_off : 0, static_cast<size_t>(NB) * es, CSZ);
        // Forward transforms read only the stored half (m < H); inverse ones
        // read the whole line.
        constexpr int nload = (MODE == Y_INV) ? E : H;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if constexpr (NT) v[m] = m < nload ? ld_nt(&lane[m]) : cx<T>{T(0), T(0)};
            else v[m] = m < nload ? lane[m] : cx<T>{T(0), T(0)};
        }
        if constexpr (MODE == Y_FWD) {
            FFT_F::template run<K>(v, ax, lds, ldsw, twl, c, t);
        } else if constexpr (MODE == Y_INV) {
            FFT_I::template run<K>(v, ax, lds, ldsw, twl, c, t);
        } else {
            // Spectrum values for this thread's kz positions, fetched with the line
            // so that both memory latencies overlap.  G~ is even in ky and kz: octant
            // index min(k, 2n - k); for position P = t + NB*m that is t + NB*m when
            // m < H and NB*(E - m) - t otherwise.
            const int kyo = ky <= ny ? ky : 2 * ny - ky;
            const void *Garr = nyq ? pl.Gn : pl.G;
            const size_t gb = nyq ? static_cast<size_t>(kyo) : static_cast<size_t>(kyo) * nx + kx;
            const size_t gs = nyq ? static_cast<size_t>(ny + 1) : static_cast<size_t>(ny + 1) * nx;
            const size_t RS = sizeof(T);
            // positions t + NB*m (m < H) from glane, NB*(E - m) - t (m >= H) from
            // ghane; an inactive line reads in-bounds dummies from offset 0
            const gbl<const char> *gbase = as_global(static_cast<const char *>(Garr));
            const size_t glane = active ? (gb + t * gs) * RS : 0, ghane = active ? (gb + (NB - t) * gs) * RS : 0;
            const size_t gstep = static_cast<size_t>(NB) * gs * RS;
            T gv[E];
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const size_t idx = m < H ? m : E - m - 1;
                if constexpr (OFF32) {
                    const uint32_t o = static_cast<uint32_t>(m < H ? glane : ghane) +
                                       static_cast<uint32_t>(idx) * static_cast<uint32_t>(gstep);
                    gv[m] = *reinterpret_cast<const gbl<T> *>(gbase + o);
                } else {
                    gv[m] = *reinterpret_cast<const gbl<T> *>(gbase + (m < H ? glane : ghane) + idx * gstep);
                }
            }
            FFT_F::template run<K>(v, ax, lds, ldsw, twl, c, t);
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = scale(v[m], gv[m]);
            FFT_I::template run<K>(v, ax, lds, ldsw, twl, c, t);
        }
        // Inverse transforms keep only the first half (m < H).
        constexpr int nstore = (MODE == Y_FWD) ? E : H;
        if (active) {
#pragma unroll
            for (int m = 0; m < nstore; ++m) {
                if constexpr (NT) st_nt(&lane[m], v[m]);
                else lane[m] = v[m];
            }
        }
    }
}

// ------------------------------------------- tile order of persistent kernels --
// The hardware hands workgroup b of a launch to XCD b mod 8, and each XCD has
// its own L2.  With CHUNK and a grid that is a multiple of 8, the tiles are
// dealt to the XCDs in chunks of kTileChunk neighbours (chunk k to XCD k mod 8),
// and the workgroups of one XCD walk its chunks in order: tiles that neighbour
// in memory (column tiles sharing 128-byte lines, z tiles of mirror rows
// sharing a spectrum slice) are then in flight on one XCD and meet in its L2,
// while the XCDs together still sweep one narrow address window at a time.
// Otherwise the walk is b, b + grid, ...  The tile index grows along a
// workgroup's walk, so the first tile at or past the end ends it.  A launch
// whose workgroups take one tile each pads its grid to whole rounds of
// 8 * kTileChunk workgroups, over which the chunked order is one to one.
//
// Measured on single solves: the chunked order takes the 1152^3 FP32 solve
// from 139 to 114 ms (its forward y pass from 36 to 16 ms) and 576^3 / 768^3
// 3-4 % lower, but slows the power-of-two lines of 512^3 (1024-point y passes
// 2 % in FP32, 6 % in FP64), so the 16-family keeps the round-robin order.
constexpr int kTileChunk = 8;
struct TileWalk {
    int i, step, x;  // x < 0: the tile is i itself
    __device__ __forceinline__ int tile() const {
        return x < 0 ? i : ((i / kTileChunk) * 8 + x) * kTileChunk + i % kTileChunk;
    }
};
template <bool CHUNK>
__device__ __forceinline__ TileWalk tile_walk() {
    const int G = static_cast<int>(gridDim.x), b = static_cast<int>(blockIdx.x);
    if (!CHUNK || G < 8 || (G & 7) != 0) return TileWalk{b, G, -1};
    return TileWalk{b >> 3, G >> 3, b & 7};
}

// ------------------------------------------------ persistent z convolution --
// Store of one complex value through a raw buffer resource: a store at or past
// `bytes` is dropped by the hardware's range check, so lanes without a line
// store nothing without a branch around the store.
// NT: a nontemporal store (cache-policy bit 1).
template <typename T, bool NT = false>
__device__ __forceinline__ void buffer_store(const cx<T> v, char *base, uint32_t bytes, uint32_t off) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, static_cast<short>(0),
                                                                        static_cast<int>(bytes), 0x00020000);
    if constexpr (sizeof(T) == 4) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, off, 0, NT ? 2 : 0);
    } else {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), rs, off, 0, NT ? 2 : 0);
    }
}

// One z line of a compile-time Z_CONV launch for lane (c, t) of the tile that
// virtual workgroup `bid` handles: the same decomposition as pass_kernel's.
// WIDE (z lines of arrays of 4 GB or more): 64-bit bases per position block
// (LinePtrW), `bytes` is the position stride (a lane's offset stays below it),
// and g points at the line's own spectrum run.
template <typename T, bool WIDE = false>
struct ZLine {
    std::conditional_t<WIDE, LinePtrW<T>, LinePtr<T, true>> lane;  // positions t + NB*m in W (or Wn)
    const gbl<const char> *g;  // spectrum octant (G, or Gn for the Nyquist column)
    uint32_t glo, ghi, gstep;  // byte offsets of positions t + NB*m (m < E/2) and NB*(E-m) - t
    uint32_t bytes;            // size of the line's array (W or Wn)
    int active;
};

// GZ: the spectrum is stored kz-fastest (octant index (kyo*nx + kx)*(nz+1) + kz,
// Nyquist column kyo*(nz+1) + kz), for lanes that walk along a line.
template <typename T, int E, int NB, int TILE, bool GZ = false, bool WIDE = false>
__device__ __forceinline__ ZLine<T, WIDE> z_line(const LaunchArgs &args, int bid, int c, int t) {
    constexpr int CSZ = static_cast<int>(sizeof(cx<T>));
    int sgi = 0;
    while (sgi + 1 < args.nseg && bid >= args.seg[sgi + 1].wg_begin) ++sgi;
    const Segment &sg = args.seg[sgi];
    int local = bid - sg.wg_begin;
    const int member = local % sg.group;
    local /= sg.group;
    const ProbArg &pa = args.p[sg.first + member];
    // The plan is read through the constant address space: it does not change
    // during the launch, so its fields come in scalar loads even after the
    // stores of an earlier tile (a vector load there would wait for them).
    using cplan = const __attribute__((address_space(4))) DevPlan;
    const auto &pl = *(cplan *)pa.plan;
    const int nx = pl.nx, ny = pl.ny;
    const bool nyq = local >= sg.wg_main;
    if (nyq) local -= sg.wg_main;
    const int g = local * TILE + c;
    ZLine<T, WIDE> zl;
    int ky, kx;
    size_t lane_off;
    const void *arr;
    if (!nyq) {
        // rows of the plane in the order 0, 1, 2ny-1, 2, 2ny-2, ..., ny: ky and its
        // mirror (same spectrum values) go to neighbouring tiles
        zl.active = g < 2 * ny * nx;
        const int vrow = zl.active ? g / nx : 0;
        kx = g - vrow * nx;
        ky = vrow == 0 ? 0 : (vrow == 2 * ny - 1 ? ny : ((vrow & 1) ? (vrow + 1) >> 1 : 2 * ny - (vrow >> 1)));
        arr = pa.W;
        // z = t + NB*m sits in tile z/zb at row z%zb; zb divides NB
        const int zb = pl.zb;
        const int sh = __builtin_ctz(static_cast<unsigned>(zb));
        lane_off = static_cast<size_t>(ky) * zb * nx + kx +
                   (static_cast<size_t>(t >> sh) * 2 * ny * zb + (t & (zb - 1))) * nx;
        if constexpr (WIDE) {
            zl.lane = LinePtrW<T>{const_cast<char *>(static_cast<const char *>(arr)),
                                  (zl.active ? lane_off : 0) * CSZ, static_cast<size_t>(NB) * 2 * ny * nx * CSZ};
            zl.bytes = static_cast<uint32_t>(zl.lane.step);
        } else {
            zl.lane = line_ptr<T, true>(arr, zl.active ? lane_off : 0, static_cast<size_t>(NB) * 2 * ny * nx, CSZ);
            zl.bytes = static_cast<uint32_t>(static_cast<size_t>(pl.nz) * 2 * ny * nx * CSZ);
        }
    } else {
        zl.active = g < 2 * ny;
        ky = g;
        kx = nx;
        arr = pa.Wn;
        lane_off = static_cast<size_t>(g) + static_cast<size_t>(t) * 2 * ny;
        if constexpr (WIDE) {
            zl.lane = LinePtrW<T>{const_cast<char *>(static_cast<const char *>(arr)),
                                  (zl.active ? lane_off : 0) * CSZ, static_cast<size_t>(NB) * 2 * ny * CSZ};
            zl.bytes = static_cast<uint32_t>(zl.lane.step);
        } else {
            zl.lane = line_ptr<T, true>(arr, zl.active ? lane_off : 0, static_cast<size_t>(NB) * 2 * ny, CSZ);
            zl.bytes = static_cast<uint32_t>(static_cast<size_t>(pl.nz) * 2 * ny * CSZ);
        }
    }
    // G~ is even in ky and kz: octant index min(k, 2n - k)
    const int kyo = ky <= ny ? ky : 2 * ny - ky;
    zl.g = as_global(static_cast<const char *>(nyq ? pl.Gn : pl.G));
    size_t gb, gs;
    if constexpr (GZ) {
        gb = (nyq ? static_cast<size_t>(kyo) : static_cast<size_t>(kyo) * nx + kx) * (pl.nz + 1);
        gs = 1;
    } else {
        gb = nyq ? static_cast<size_t>(kyo) : static_cast<size_t>(kyo) * nx + kx;
        gs = nyq ? static_cast<size_t>(ny + 1) : static_cast<size_t>(ny + 1) * nx;
    }
    if constexpr (WIDE && GZ) {
        // the line's own run of the spectrum: offsets within it stay small
        if (zl.active) zl.g += gb * sizeof(T);
        gb = 0;
    }
    zl.glo = zl.active ? static_cast<uint32_t>((gb + t * gs) * sizeof(T)) : 0u;
    zl.ghi = zl.active ? static_cast<uint32_t>((gb + (NB - t) * gs) * sizeof(T)) : 0u;
    zl.gstep = static_cast<uint32_t>(static_cast<size_t>(NB) * gs * sizeof(T));
    return zl;
}

// One y line of a compile-time Y_FWD / Y_INV launch for lane (c, t) of the
// tile that virtual workgroup `bid` handles: line (z, kx) has position y at
// w_row(z, y) + kx; the Nyquist line of plane z is contiguous in Wn.  No
// spectrum (g stays null).
template <typename T, int NB, int TILE>
__device__ __forceinline__ ZLine<T> y_line(const LaunchArgs &args, int bid, int c, int t) {
    constexpr int CSZ = static_cast<int>(sizeof(cx<T>));
    int sgi = 0;
    while (sgi + 1 < args.nseg && bid >= args.seg[sgi + 1].wg_begin) ++sgi;
    const Segment &sg = args.seg[sgi];
    int local = bid - sg.wg_begin;
    const int member = local % sg.group;
    local /= sg.group;
    const ProbArg &pa = args.p[sg.first + member];
    using cplan = const __attribute__((address_space(4))) DevPlan;
    const auto &pl = *(cplan *)pa.plan;
    const int nx = pl.nx, ny = pl.ny, nz = pl.nz;
    const bool nyq = local >= sg.wg_main;
    if (nyq) local -= sg.wg_main;
    const int g = local * TILE + c;
    ZLine<T> yl;
    if (!nyq) {
        yl.active = g < nz * nx;
        const int z = yl.active ? g / nx : 0;
        const int kx = g - z * nx;
        const size_t es = static_cast<size_t>(pl.zb) * nx;
        const size_t lane_off = w_row(z, 0, ny, nx, pl.zb) + kx + static_cast<size_t>(t) * es;
        yl.lane = line_ptr<T, true>(pa.W, yl.active ? lane_off : 0, NB * es, CSZ);
        yl.bytes = static_cast<uint32_t>(static_cast<size_t>(nz) * 2 * ny * nx * CSZ);
    } else {
        yl.active = g < nz;
        const size_t lane_off = static_cast<size_t>(g) * 2 * ny + t;
        yl.lane = line_ptr<T, true>(pa.Wn, yl.active ? lane_off : 0, NB, CSZ);
        yl.bytes = static_cast<uint32_t>(static_cast<size_t>(nz) * 2 * ny * CSZ);
    }
    yl.g = nullptr;
    yl.glo = yl.ghi = yl.gstep = 0u;
    return yl;
}

// Column passes (Y_FWD, Z_CONV, Y_INV) for lines of 16, 32 or 64 threads
// (ST = 3: radices E, M, K with M*K = NB; ST = 4: E, M, M, K with M*M*K = NB,
// FP32 only; a tile of wave_tile() lines): each line lies within one wavefront
// (wavefront w holds lines w*64/NB onwards), so the stage exchanges stay inside
// the wavefront and need no workgroup barrier.  The tile's stored half (all of
// it for Y_INV) is loaded with adjacent lanes on adjacent lines (128-byte row
// segments) and transposed through each line's LDS row; the results (the
// stored half, all of them for Y_FWD) go back the same way.  Z_CONV: the
// spectrum is stored kz-fastest for such plans, so each line's values are read
// in contiguous runs.
//
// PERSIST: the workgroup walks its tiles (tile_walk) and issues the next
// tile's line (and spectrum) loads before the current tile's stores.  Vector
// loads and stores retire in order, so a load issued after stores cannot be
// waited for without waiting for them; issued first, the loads run under the
// current tile's transforms and no wait covers the stores.  For the compiler's
// wait counts to be exact, every load and store of a pass through the loop is
// unconditional (the last tile loads its own line again; lanes without a line
// store past the end of the array, which the buffer range check drops), the
// loop is entered with nothing outstanding, and plan fields are read through
// the constant address space (scalar loads; a vector load there would wait for
// the previous tile's stores).  Otherwise the workgroup takes one tile.
template <typename T, int E, int K, int MODE, bool PERSIST, int ST = 3, bool WIDE = false, bool NT = false>
__global__ void __launch_bounds__((max_block_for(sizeof(T) == 4 ? 0 : 1, E)))
__attribute__((amdgpu_waves_per_eu(wave_waves_per_simd(sizeof(T) == 4 ? 0 : 1, MODE, E,
                                                       wave_nb(E, K, ST), ST))))
wave_col_kernel(const LaunchArgs args) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem);
    static_assert(MODE == Y_FWD || MODE == Z_CONV || MODE == Y_INV, "column passes");
    static_assert(ST == 3 || (ST == 4 && sizeof(T) == 4), "three-stage lines, or four-stage ones in FP32");
    static_assert(!WIDE || MODE == Z_CONV, "64-bit bases for z lines only");
    constexpr int H = E / 2;
    constexpr int NB = wave_nb(E, K, ST);
    static_assert(NB == 16 || NB == 32 || NB == 64, "lines of 16, 32 or 64 threads");
    constexpr int L = E * NB;
    constexpr int TILE = wave_tile(sizeof(T) == 4 ? 0 : 1, MODE, E, NB, ST);
    constexpr int S = wave_line_stride(L);
    constexpr int NLOAD = MODE == Y_INV ? E : H;   // forward transforms read the stored half
    constexpr int NSTORE = MODE == Y_FWD ? E : H;  // inverse ones keep the first half
    constexpr bool ZC = MODE == Z_CONV;
    using FFT_F = LineFFT<T, E, -1, true, NB, S>;
    using FFT_I = LineFFT<T, E, +1, true, NB, S>;

    // (one tile per workgroup: the launch pads its grid to a multiple of 64, so
    // that the chunked order maps the workgroups onto the tiles one to one)
    TileWalk walk = tile_walk<E != 16>();
    int bid = walk.tile();
    if (bid >= args.nwg) return;
    const int tid = threadIdx.x;
    const int cc = tid & (TILE - 1), tc = tid >> __builtin_ctz(TILE);  // adjacent lanes on adjacent lines
    const int cw = tid >> __builtin_ctz(NB), tw = tid & (NB - 1);       // line cw lies in one wavefront
    const AxisPlan &ax0 = args.p[0].plan->ax[ZC ? 2 : 1];
    constexpr bool TWL = wave_tw_lds(sizeof(T) == 4 ? 0 : 1, MODE, E, NB, ST);
    const auto twl = [&]() __attribute__((always_inline)) {
        if constexpr (TWL) {
            cx<T> *p = lds + TILE * S;
            copy_to_lds<T>(p, ax0.tw, ax0.ntw);  // published by the first barrier below
            return static_cast<const cx<T> *>(p);
        } else {
            return as_global(static_cast<const cx<T> *>(ax0.tw));
        }
    }();
    // position P = t + NB*m of a line's row sits at P + P/16 = t + t/16 + m*(NB + NB/16)
    constexpr int RM = NB + NB / 16;
    cx<T> *rowc = lds + cc * S + tc + (tc >> 4);
    cx<T> *roww = lds + cw * S + tw + (tw >> 4);

    auto line = [&](int b) __attribute__((always_inline)) {
        if constexpr (ZC) return z_line<T, E, NB, TILE, false, WIDE>(args, b, cc, tc);
        else return y_line<T, NB, TILE>(args, b, cc, tc);
    };
    auto load_g = [&](int b, T *gv) __attribute__((always_inline)) {
        if constexpr (ZC) {
            const ZLine<T, WIDE> zl = z_line<T, E, NB, TILE, true, WIDE>(args, b, cw, tw);
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const uint32_t idx = m < H ? m : E - m - 1;
                gv[m] = *reinterpret_cast<const gbl<T> *>(zl.g + ((m < H ? zl.glo : zl.ghi) + idx * zl.gstep));
            }
        }
    };
    auto cur = line(bid);
    T gnx[ZC ? E : 1];
    if constexpr (sizeof(T) == 4) {
        // the line first (loads retire in order: its rows can be written
        // while the spectrum values are still in flight)
        cx<T> first[NLOAD];
#pragma unroll
        for (int m = 0; m < NLOAD; ++m) first[m] = NT ? ld_nt(&cur.lane[m]) : cur.lane[m];
        load_g(bid, gnx);
#pragma unroll
        for (int m = 0; m < NLOAD; ++m) rowc[m * RM] = first[m];
    } else {
        // FP64: sixteen-byte values held there do not stay in registers
        load_g(bid, gnx);
#pragma unroll
        for (int m = 0; m < NLOAD; ++m) rowc[m * RM] = NT ? ld_nt(&cur.lane[m]) : cur.lane[m];
    }
    if constexpr (PERSIST) __builtin_amdgcn_s_waitcnt(0x0f70);  // nothing outstanding on entry (vmcnt 0)
    for (;;) {
        __syncthreads();  // the tile is in the rows (and, first time, the twiddles)
        cx<T> v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = m < NLOAD ? roww[m * RM] : cx<T>{T(0), T(0)};
        if constexpr (MODE != Y_INV) FFT_F::template run<K, true, true>(v, ax0, lds, S, twl, cw, tw);
        if constexpr (ZC) {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = scale(v[m], gnx[m]);
        }
        // the next tile's line (and spectrum values), before this tile's stores
        walk.i += walk.step;
        const int nbid = walk.tile();
        const bool more = PERSIST && nbid < args.nwg;
        const int fbid = more ? nbid : bid;
        // FP64: the line is loaded after this tile's stores (the extra 16-byte
        // values held across the inverse transform do not stay in registers)
        constexpr bool PF = PERSIST && sizeof(T) == 4;
        auto fol = cur;
        cx<T> nxt[PF ? NLOAD : 1];
        if constexpr (PERSIST) {
            fol = line(fbid);
            if constexpr (PF) {
#pragma unroll
                for (int m = 0; m < NLOAD; ++m) nxt[m] = NT ? ld_nt(&fol.lane[m]) : fol.lane[m];
            }
            load_g(fbid, gnx);
        }
        (void)nxt;
        if constexpr (MODE != Y_FWD) FFT_I::template run<K, true, true>(v, ax0, lds, S, twl, cw, tw);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int m = 0; m < NSTORE; ++m) roww[m * RM] = v[m];
        __syncthreads();  // results are in the rows
#pragma unroll
        for (int m = 0; m < NSTORE; ++m) {
            if constexpr (WIDE) {
                buffer_store<T, NT>(rowc[m * RM], cur.lane.block(m), cur.bytes,
                                    cur.active ? static_cast<uint32_t>(cur.lane.lane) : 0xfffffff0u);
            } else {
                const uint32_t off = static_cast<uint32_t>(cur.lane.lane) +
                                     static_cast<uint32_t>(m) * static_cast<uint32_t>(cur.lane.step);
                buffer_store<T, NT>(rowc[m * RM], cur.lane.base, cur.bytes, cur.active ? off : 0xfffffff0u);
            }
        }
        if (!more) break;
        __syncthreads();  // the rows have been read
        if constexpr (PF) {
#pragma unroll
            for (int m = 0; m < NLOAD; ++m) rowc[m * RM] = nxt[m];
        } else {
#pragma unroll
            for (int m = 0; m < NLOAD; ++m) rowc[m * RM] = NT ? ld_nt(&fol.lane[m]) : fol.lane[m];
        }
        cur = fol;
        bid = nbid;
    }
}

// ------------------------------------------------- persistent column passes --
// Column passes (Y_FWD, Z_CONV, Y_INV) with compile-time lines where one
// workgroup of the column kernel fills a compute unit (long lines; FP64 from
// 1024 points): the workgroup walks its tiles (tile_walk) and loads the
// next tile's line (and spectrum values) after the current tile's forward
// transform and before its stores, so those loads run under the rest of the
// work and no wait covers the stores (loads and stores retire in order).  For
// the compiler's wait counts to be exact every load and store of the loop is
// unconditional: a lane past the last line of its set takes that line again
// (the same values go to the same addresses), the last tile prefetches itself,
// and the loop is entered with nothing outstanding.
template <typename T, bool OFF32>
struct ColLine {
    LinePtr<T, OFF32> lane;  // positions t + NB*m of the line in W (or Wn)
    const char *g;           // z: spectrum octant (G, or Gn for the Nyquist column)
    size_t glo, ghi, gstep;  // z: byte offsets of positions t + NB*m (m < E/2) and NB*(E-m) - t
};

// Line of lane (c, t) of the tile that workgroup `bid` handles: the same
// decomposition as pass_kernel's.
template <typename T, int MODE, int NB, int TILE, bool OFF32>
__device__ __forceinline__ ColLine<T, OFF32> col_line(const LaunchArgs &args, int bid, int c, int t) {
    constexpr int CSZ = static_cast<int>(sizeof(cx<T>));
    int sgi = 0;
    while (sgi + 1 < args.nseg && bid >= args.seg[sgi + 1].wg_begin) ++sgi;
    const Segment &sg = args.seg[sgi];
    int local = bid - sg.wg_begin;
    const int member = local % sg.group;
    local /= sg.group;
    const ProbArg &pa = args.p[sg.first + member];
    // constant address space: scalar loads that do not wait for earlier stores
    using cplan = const __attribute__((address_space(4))) DevPlan;
    const auto &pl = *(cplan *)pa.plan;
    const int nx = pl.nx, ny = pl.ny, nz = pl.nz;
    const bool nyq = local >= sg.wg_main;
    if (nyq) local -= sg.wg_main;
    int g = local * TILE + c;
    ColLine<T, OFF32> cl;
    cl.g = nullptr;
    cl.glo = cl.ghi = cl.gstep = 0;
    if constexpr (MODE == Z_CONV) {
        int ky, kx;
        if (!nyq) {
            // rows in the order 0, 1, 2ny-1, 2, 2ny-2, ..., ny (mirror pairs in neighbouring tiles)
            g = min(g, 2 * ny * nx - 1);
            const int vrow = g / nx;
            kx = g - vrow * nx;
            ky = vrow == 0 ? 0 : (vrow == 2 * ny - 1 ? ny : ((vrow & 1) ? (vrow + 1) >> 1 : 2 * ny - (vrow >> 1)));
            // z = t + NB*m sits in tile z/zb at row z%zb; zb divides NB
            const int zb = pl.zb;
            const int sh = __builtin_ctz(static_cast<unsigned>(zb));
            const size_t off = static_cast<size_t>(ky) * zb * nx + kx +
                               (static_cast<size_t>(t >> sh) * 2 * ny * zb + (t & (zb - 1))) * nx;
            cl.lane = line_ptr<T, OFF32>(pa.W, off, static_cast<size_t>(NB) * 2 * ny * nx, CSZ);
        } else {
            g = min(g, 2 * ny - 1);
            ky = g;
            kx = nx;
            cl.lane = line_ptr<T, OFF32>(pa.Wn, static_cast<size_t>(g) + static_cast<size_t>(t) * 2 * ny,
                                         static_cast<size_t>(NB) * 2 * ny, CSZ);
        }
        // G~ is even in ky and kz: octant index min(k, 2n - k)
        const int kyo = ky <= ny ? ky : 2 * ny - ky;
        cl.g = static_cast<const char *>(nyq ? pl.Gn : pl.G);
        const size_t gb = nyq ? static_cast<size_t>(kyo) : static_cast<size_t>(kyo) * nx + kx;
        const size_t gs = nyq ? static_cast<size_t>(ny + 1) : static_cast<size_t>(ny + 1) * nx;
        cl.glo = (gb + t * gs) * sizeof(T);
        cl.ghi = (gb + (NB - t) * gs) * sizeof(T);
        cl.gstep = static_cast<size_t>(NB) * gs * sizeof(T);
    } else {
        // y lines: line (z, kx) has position y at w_row(z, y) + kx; the Nyquist
        // line of plane z is contiguous in Wn
        if (!nyq) {
            g = min(g, nz * nx - 1);
            const int z = g / nx;
            const int kx = g - z * nx;
            const size_t es = static_cast<size_t>(pl.zb) * nx;
            cl.lane = line_ptr<T, OFF32>(pa.W, w_row(z, 0, ny, nx, pl.zb) + kx + static_cast<size_t>(t) * es,
                                         static_cast<size_t>(NB) * es, CSZ);
        } else {
            g = min(g, nz - 1);
            cl.lane = line_ptr<T, OFF32>(pa.Wn, static_cast<size_t>(g) * 2 * ny + t, static_cast<size_t>(NB), CSZ);
        }
    }
    return cl;
}

template <typename T, int E, int K, int MODE, int FIX>
__global__ void __launch_bounds__((max_block_for(sizeof(T) == 4 ? 0 : 1, E))) col_persist_kernel(const LaunchArgs args) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem);
    static_assert(MODE == Y_FWD || MODE == Z_CONV || MODE == Y_INV, "column passes");
    constexpr int prec = sizeof(T) == 4 ? 0 : 1;
    constexpr int ST = fix_stages(FIX);
    static_assert(ST >= 2 && ST <= 4, "compile-time lines");
    constexpr bool OFF32 = fix_off32(FIX);
    constexpr bool ZC = MODE == Z_CONV;
    constexpr int H = E / 2;
    constexpr int NLOAD = MODE == Y_INV ? E : H;   // forward transforms read the stored half
    constexpr int NSTORE = MODE == Y_FWD ? E : H;  // inverse ones keep the first half
    constexpr int CSZ = static_cast<int>(sizeof(cx<T>));
    constexpr int NB = fix_nb(FIX, E, K);
    constexpr int TILE = pass_tile(prec, MODE, E, NB);
    constexpr int L = E * NB;
    constexpr int LDSW = col_ldsw(prec, MODE, E, NB);
    constexpr bool GT = col_tables_global(prec, MODE, E, NB);  // twiddles in global memory
    using FFT_F = LineFFT<T, E, -1, false, NB, LDSW>;
    using FFT_I = LineFFT<T, E, +1, false, NB, LDSW>;

    TileWalk walk = tile_walk<E != 16>();
    int bid = walk.tile();
    if (bid >= args.nwg) return;
    const int tid = threadIdx.x;
    const int c = tid & (TILE - 1), t = tid >> __builtin_ctz(TILE);  // adjacent lanes on adjacent lines
    // every problem of the launch has lines of length L: the same stage twiddles
    const AxisPlan &ax0 = args.p[0].plan->ax[ZC ? 2 : 1];
    const auto twl = [&]() __attribute__((always_inline)) {
        if constexpr (GT) {
            return as_global(static_cast<const cx<T> *>(ax0.tw));
        } else {
            cx<T> *p = lds + L * LDSW;
            copy_to_lds<T>(p, ax0.tw, ax0.ntw);  // published by the first transform's barrier
            return static_cast<const cx<T> *>(p);
        }
    }();

    cx<T> ln[NLOAD];     // the loaded part of this thread's line
    T gn[ZC ? E : 1];    // z: spectrum values of its positions
    auto load = [&](const ColLine<T, OFF32> &cl) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < NLOAD; ++m) ln[m] = cl.lane[m];
        if constexpr (ZC) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const size_t idx = m < H ? m : E - m - 1;
                const size_t o = (m < H ? cl.glo : cl.ghi) + idx * cl.gstep;
                if constexpr (OFF32)
                    gn[m] = *reinterpret_cast<const gbl<T> *>(as_global(cl.g) + static_cast<uint32_t>(o));
                else
                    gn[m] = *reinterpret_cast<const gbl<T> *>(as_global(cl.g) + o);
            }
        }
    };
    ColLine<T, OFF32> cur = col_line<T, MODE, NB, TILE, OFF32>(args, bid, c, t);
    load(cur);
    __builtin_amdgcn_s_waitcnt(0x0f70);  // nothing outstanding on entry (vmcnt 0)
    for (;;) {
        cx<T> v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = m < NLOAD ? ln[m] : cx<T>{T(0), T(0)};
        // the next tile's line (and spectrum values), before this tile's stores:
        // y passes issue it before their transform, the z pass after the forward
        // transform (the spectrum values of this tile are needed up to there)
        walk.i += walk.step;
        const int nbid = walk.tile();
        const bool more = nbid < args.nwg;
        const ColLine<T, OFF32> nxt = col_line<T, MODE, NB, TILE, OFF32>(args, more ? nbid : bid, c, t);
        if constexpr (!ZC) load(nxt);
        // the first barrier of the first transform retires the last tile's LDS readers
        if constexpr (MODE != Y_INV) FFT_F::template run<K>(v, ax0, lds, LDSW, twl, c, t);
        if constexpr (ZC) {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = scale(v[m], gn[m]);
            load(nxt);
        }
        if constexpr (MODE != Y_FWD) FFT_I::template run<K>(v, ax0, lds, LDSW, twl, c, t);
#pragma unroll
        for (int m = 0; m < NSTORE; ++m) cur.lane[m] = v[m];
        if (!more) break;
        cur = nxt;
        bid = nbid;
    }
}

// Where the column kernels run persistently (PSPFFT_COL_PERSIST: 0 never,
// 1 always, unset: where one workgroup fills a compute unit).
inline int col_persist_mode() {
    static int v = -2;
    if (v == -2) {
        v = -1;
        if (const char *e = std::getenv("PSPFFT_COL_PERSIST")) v = std::atoi(e) != 0 ? 1 : 0;
    }
    return v;
}

template <typename T, int E, int K, int MODE, int FIX>
hipError_t launch_col(const LaunchArgs &args, int grid, int block, size_t lds, hipStream_t stream) {
    constexpr int kMaxDevices = 64;
    static int per_cu[kMaxDevices] = {0}, cus[kMaxDevices] = {0};
    static size_t seen_lds[kMaxDevices] = {0};
    auto fo = pass_kernel<T, E, K, MODE, FIX>;
    auto fp = col_persist_kernel<T, E, K, MODE, FIX>;
    // z lines of a streaming launch: nontemporal line loads and stores
    auto fs = pass_kernel<T, E, K, MODE, FIX, MODE == Z_CONV>;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (per_cu[dev] == 0 || seen_lds[dev] != lds) {
        for (auto f : {fo, fp, fs}) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    160 * 1024);
            if (e != hipSuccess) return e;
        }
        int p = 0, c = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&p, fo, block, lds);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        per_cu[dev] = p > 0 ? p : 1;
        cus[dev] = c > 0 ? c : 1;
        seen_lds[dev] = lds;
    }
    // Measured: the y passes gain where a tile's row segment is a whole
    // 128-byte line or the values are FP32, and lose a third with FP64 tiles of
    // 64-byte segments (lines of 2048), whose pairs of tiles share lines that
    // long-lived workgroups no longer fetch at nearly the same time.
    constexpr int prec = sizeof(T) == 4 ? 0 : 1;
    constexpr int NB = fix_nb(FIX, E, K);
    constexpr bool y_ok = MODE == Z_CONV || prec == 0 ||
                          pass_tile(prec, MODE, E, NB) * static_cast<int>(sizeof(cx<T>)) >= 128;
    const int mode = col_persist_mode();
    if (mode == 1 || (mode < 0 && y_ok && per_cu[dev] == 1)) {
        int g = per_cu[dev] * cus[dev];
        if (g > args.nwg) g = args.nwg;
        hipLaunchKernelGGL(fp, dim3(g), dim3(block), lds, stream, args);
    } else {
        hipLaunchKernelGGL(args.nt ? fs : fo, dim3(grid), dim3(block), lds, stream, args);
    }
    return hipGetLastError();
}

inline int zconv_persist_mode();

// The wavefront-owned column kernel: persistent where one workgroup fills a
// compute unit (zconv_persist_mode), otherwise one tile per workgroup.
template <typename T, int E, int K, int MODE, int ST = 3, bool WIDE = false>
hipError_t launch_wave_col(const LaunchArgs &args, hipStream_t stream) {
    constexpr int kMaxDevices = 64;
    constexpr int prec = sizeof(T) == 4 ? 0 : 1;
    constexpr int NB = wave_nb(E, K, ST);
    constexpr int block = wave_tile(prec, MODE, E, NB, ST) * NB;
    constexpr size_t lds = wave_lds_bytes(prec, MODE, E, NB, ST);
    static_assert(lds <= 160 * 1024, "tile rows and twiddles fit the LDS");
    static int per_cu[kMaxDevices] = {0}, cus[kMaxDevices] = {0};
    auto fp = wave_col_kernel<T, E, K, MODE, true, ST, WIDE>;
    auto fo = wave_col_kernel<T, E, K, MODE, false, ST, WIDE>;
    // FP32 z lines below 4 GB of a streaming launch: nontemporal line loads and stores
    constexpr bool NTZ = MODE == Z_CONV && sizeof(T) == 4 && !WIDE;
    auto fpn = wave_col_kernel<T, E, K, MODE, true, ST, WIDE, NTZ>;
    auto fon = wave_col_kernel<T, E, K, MODE, false, ST, WIDE, NTZ>;
    const bool nt = NTZ && args.nt;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (per_cu[dev] == 0) {
        for (auto f : {fp, fo, fpn, fon}) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    160 * 1024);
            if (e != hipSuccess) return e;
        }
        int p = 0, c = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&p, fp, block, lds);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        per_cu[dev] = p > 0 ? p : 1;
        cus[dev] = c > 0 ? c : 1;
    }
    const int mode = zconv_persist_mode();
    if (mode == 1 || (mode < 0 && per_cu[dev] == 1)) {
        int grid = per_cu[dev] * cus[dev];
        if (grid > args.nwg) grid = args.nwg;
        hipLaunchKernelGGL(nt ? fpn : fp, dim3(grid), dim3(block), lds, stream, args);
    } else {
        // chunked tile order (tile_walk): a grid of whole chunk rounds (8 XCDs x kTileChunk)
        constexpr int round = E != 16 ? 8 * kTileChunk : 1;
        const int grid = (args.nwg + round - 1) / round * round;
        hipLaunchKernelGGL(nt ? fon : fo, dim3(grid), dim3(block), lds, stream, args);
    }
    return hipGetLastError();
}

// The y passes take wavefront-owned lines (three stages, 32 or 64 threads per
// line) where the column kernel's tile needs more LDS than this, so that a CU
// holds only one of its workgroups (PSPFFT_WAVE_Y_LDS overrides, in bytes;
// 0 always).  Measured, with two or more per CU the column kernel is as fast.
inline size_t wave_y_min_lds() {
    static long v = -1;
    if (v < 0) {
        long x = 80 * 1024;
        if (const char *e = std::getenv("PSPFFT_WAVE_Y_LDS")) x = std::atol(e);
        v = x >= 0 ? x : 80 * 1024;
    }
    return static_cast<size_t>(v);
}

// Where the wavefront-owned column kernel runs persistently
// (PSPFFT_ZCONV_PERSIST: 0 never, 1 always, unset: where one workgroup fills a
// compute unit).  With two or more workgroups per unit the hardware already
// overlaps one's memory traffic with another's transforms, and its in-order
// dispatch keeps the tiles in flight neighbours in memory, which long-lived
// workgroups drift away from.
inline int zconv_persist_mode() {
    static int v = -2;
    if (v == -2) {
        v = -1;
        if (const char *e = std::getenv("PSPFFT_ZCONV_PERSIST")) v = std::atoi(e) != 0 ? 1 : 0;
    }
    return v;
}

template <typename T, int E, int K, int MODE, int FIX>
hipError_t launch_kernel(const LaunchArgs &args, int grid, int block, size_t lds, hipStream_t stream) {
    static bool attr_set = false;
    auto fn = pass_kernel<T, E, K, MODE, FIX>;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, stream, args);
    return hipGetLastError();
}

// The wavefront-owned column kernel exists for three-stage lines of 16, 32 or 64
// threads and four-stage FP32 lines of 32 or 64 threads whose tile of
// wave_tile() lines fits the family's largest workgroup and the LDS.
template <typename T, int E, int K, int MODE, int ST = 3>
constexpr bool wave_col_fits() {
    constexpr int prec = sizeof(T) == 4 ? 0 : 1;
    constexpr int M = E & -E;
    if constexpr (ST == 4) {
        constexpr int NB = wave_nb(E, K, ST);
        return prec == 0 && M < E && (NB == 32 || NB == 64) &&
               wave_tile(prec, MODE, E, NB, ST) * NB <= max_block_for(prec, E) &&
               wave_lds_bytes(prec, MODE, E, NB, ST) <= 160 * 1024;
    } else {
        constexpr int NB = M * K;
        return (NB == 16 || NB == 32 || NB == 64) && wave_tile(prec, MODE, E, NB) * NB <= max_block_for(prec, E) &&
               wave_lds_bytes(prec, MODE, E, NB) <= 160 * 1024;
    }
}

// The y passes take the wavefront-owned kernel where its tile equals the
// column kernel's (pass_tile), from which the host counted the launch's tiles:
// three-stage lines whose default tile fits the family's largest workgroup,
// and four-stage lines where the kernel runs two workgroups per CU (twiddles
// in global memory: the 36-family).  Measured, 576^3 FP32 (1152-point lines):
// y passes 1.53 / 1.77 -> 1.47 / 1.56 ms; with one workgroup per CU (the
// 20-family's 640-point lines of 320^3) 0.176 / 0.199 -> 0.215 / 0.213 ms.
template <typename T, int E, int K, int MODE, int ST>
constexpr bool wave_y_fits() {
    constexpr int prec = sizeof(T) == 4 ? 0 : 1;
    constexpr int NB = wave_nb(E, K, ST);
    return (NB == 32 || NB == 64) && wave_col_fits<T, E, K, MODE, ST>() &&
           ((ST == 3 && fix_tile(prec, MODE, NB) * NB <= max_block_for(prec, E)) ||
            (ST == 4 && !wave_tw_lds(prec, MODE, E, NB, ST))) &&
           wave_tile(prec, MODE, E, NB, ST) == pass_tile(prec, MODE, E, NB);
}

template <typename T, int E, int K, int FIX>
hipError_t launch_mode(int mode, const LaunchArgs &args, int grid, int block, size_t lds, hipStream_t stream) {
    switch (mode) {
        case X_FWD: return launch_kernel<T, E, K, X_FWD, FIX>(args, grid, block, lds, stream);
        case Y_FWD:
            if constexpr (FIX == 3 && wave_y_fits<T, E, K, Y_FWD, 3>()) {
                if (col_default_lds(sizeof(T) == 4 ? 0 : 1, Y_FWD, E, wave_nb(E, K, 3)) > wave_y_min_lds())
                    return launch_wave_col<T, E, K, Y_FWD>(args, stream);
            }
            if constexpr (FIX == 4 && wave_y_fits<T, E, K, Y_FWD, 4>()) {
                if (col_default_lds(sizeof(T) == 4 ? 0 : 1, Y_FWD, E, wave_nb(E, K, 4)) > wave_y_min_lds())
                    return launch_wave_col<T, E, K, Y_FWD, 4>(args, stream);
            }
            if constexpr (FIX != 0) return launch_col<T, E, K, Y_FWD, FIX>(args, grid, block, lds, stream);
            else return launch_kernel<T, E, K, Y_FWD, FIX>(args, grid, block, lds, stream);
        case Z_CONV:
            if constexpr (FIX == 3 && wave_col_fits<T, E, K, Z_CONV>()) {
                if (args.wave_z) return launch_wave_col<T, E, K, Z_CONV>(args, stream);
            }
            if constexpr (FIX == 4 && wave_col_fits<T, E, K, Z_CONV, 4>()) {
                if (args.wave_z) return launch_wave_col<T, E, K, Z_CONV, 4>(args, stream);
            }
            if constexpr (FIX == 3 + kFixWide && wave_col_fits<T, E, K, Z_CONV>()) {
                if (args.wave_z) return launch_wave_col<T, E, K, Z_CONV, 3, true>(args, stream);
            }
            if constexpr (FIX == 4 + kFixWide && wave_col_fits<T, E, K, Z_CONV, 4>()) {
                if (args.wave_z) return launch_wave_col<T, E, K, Z_CONV, 4, true>(args, stream);
            }
            if (args.wave_z) return hipErrorInvalidValue;  // a kz-fastest spectrum needs wave_col_kernel
            if constexpr (FIX != 0) return launch_col<T, E, K, Z_CONV, FIX>(args, grid, block, lds, stream);
            else return launch_kernel<T, E, K, Z_CONV, FIX>(args, grid, block, lds, stream);
        case Y_INV:
            if constexpr (FIX == 3 && wave_y_fits<T, E, K, Y_INV, 3>()) {
                if (col_default_lds(sizeof(T) == 4 ? 0 : 1, Y_INV, E, wave_nb(E, K, 3)) > wave_y_min_lds())
                    return launch_wave_col<T, E, K, Y_INV>(args, stream);
            }
            if constexpr (FIX == 4 && wave_y_fits<T, E, K, Y_INV, 4>()) {
                if (col_default_lds(sizeof(T) == 4 ? 0 : 1, Y_INV, E, wave_nb(E, K, 4)) > wave_y_min_lds())
                    return launch_wave_col<T, E, K, Y_INV, 4>(args, stream);
            }
            if constexpr (FIX != 0) return launch_col<T, E, K, Y_INV, FIX>(args, grid, block, lds, stream);
            else return launch_kernel<T, E, K, Y_INV, FIX>(args, grid, block, lds, stream);
        case X_INV: return launch_kernel<T, E, K, X_INV, FIX>(args, grid, block, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

// fix: 0 (run-time geometry), 2, 3 or 4 (compile-time lines of that many
// stages), plus kFixWide for 64-bit addresses.  Three- and four-stage instances
// exist where a workgroup of pass_tile() lines fits the family's largest
// workgroup; four-stage ones where such a line (E*M*M*K points) can occur.
template <typename T, int E, int K>
hipError_t launch_fix(int mode, int fix, const LaunchArgs &args, int grid, int block, size_t lds,
                      hipStream_t stream) {
    constexpr int prec = sizeof(T) == 4 ? 0 : 1;
    constexpr int M = E & -E;
    constexpr int W = kFixWide;
    if constexpr (K > 1) {
        if (fix == 2) return launch_mode<T, E, K, 2>(mode, args, grid, block, lds, stream);
        if (fix == 2 + W) return launch_mode<T, E, K, 2 + W>(mode, args, grid, block, lds, stream);
        if constexpr (pass_tile(prec, Y_FWD, E, M * K) * M * K <= max_block_for(prec, E)) {
            if (fix == 3) return launch_mode<T, E, K, 3>(mode, args, grid, block, lds, stream);
            if (fix == 3 + W) return launch_mode<T, E, K, 3 + W>(mode, args, grid, block, lds, stream);
        }
        if constexpr (M < E && E * M * M * K <= 4096 &&
                      pass_tile(prec, Y_FWD, E, M * M * K) * M * M * K <= max_block_for(prec, E)) {
            if (fix == 4) return launch_mode<T, E, K, 4>(mode, args, grid, block, lds, stream);
            if (fix == 4 + W) return launch_mode<T, E, K, 4 + W>(mode, args, grid, block, lds, stream);
        }
    }
    if (fix != 0) return hipErrorInvalidValue;
    return launch_mode<T, E, K, 0>(mode, args, grid, block, lds, stream);
}

// All last-stage radices a family can have: 1 (single stage) and the powers of
// two up to the middle radix.
template <typename T, int E>
hipError_t launch_family(int mode, int K, int fix, const LaunchArgs &args, int grid, int block, size_t lds,
                         hipStream_t stream) {
    constexpr int M = E & -E;
    switch (K) {
        case 1: return launch_fix<T, E, 1>(mode, fix, args, grid, block, lds, stream);
        case 2: return launch_fix<T, E, 2>(mode, fix, args, grid, block, lds, stream);
        case 4: return launch_fix<T, E, 4>(mode, fix, args, grid, block, lds, stream);
        case 8:
            if constexpr (M >= 8) return launch_fix<T, E, 8>(mode, fix, args, grid, block, lds, stream);
            else return hipErrorInvalidValue;
        case 16:
            if constexpr (M >= 16) return launch_fix<T, E, 16>(mode, fix, args, grid, block, lds, stream);
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pspfft
