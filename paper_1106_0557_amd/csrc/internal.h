// internal.h -- data structures shared by the HIP kernels and the host runtime.
//
// Workspace layout of one in-flight solve (complex values of the precision):
//   W  : [z / B][ky < 2ny][z % B][kx < nx]   main part in tiles of B z planes
//                                            (rows of nx values, aligned)
//   Wn : [z < nz][ky < 2ny]                  the kx = nx (Nyquist) column, split
//                                            off so that every row of W is aligned
// B (DevPlan::zb, a power of two up to 16 that divides the z lines' threads per
// line; 1 unless a z plane spans 4 MB or more) keeps the z lines of the z pass
// within nz/B regions of B rows instead of nz planes far apart, which the address
// translation caches cannot hold for large meshes.  Row (z, ky) starts at element
// ((z/B)*2ny + ky)*B*nx + (z%B)*nx.
// The x pass writes rows ky = y < ny of every z plane; the y pass fills all 2ny
// rows; the z pass works in place on z < nz; the inverse y pass leaves rows
// y < ny; the inverse x pass reads them.  The upper z half of the doubled mesh
// is never stored: it is zero on input and discarded on output.
//
// Green's-function spectrum (plan precision), octant kx <= nx, ky <= ny, kz <= nz:
//   G  : [kz][ky][kx < nx]   row stride nx
//   Gn : [kz][ky]            kx = nx
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pspfft {

constexpr int kMaxStages = 10;
constexpr int kMaxProblems = 32;  // problems per grouped launch

// One transform line along one axis, split into stages of radix R[s].
// y and z lines have length L = 2n (the doubled mesh).  x lines use the packed
// real-to-complex form: the 2n real values of a zero-padded row become n
// complex values, so L = n there, plus a split step with exp(-i pi k / n).
// A line is handled by NB = L / E threads, each owning the E positions
// t + NB*m (m < E) before the first and after the last stage; the upper half of
// the input (m >= E/2) is the zero padding and the upper half of the output is
// never needed, so both are known at compile time.
//
// Lengths outside the families (E = 0, NB = 0) run on the generic line kernel
// (line_generic.hip) with stages of radix 8, 4 or 2, then 5, 9 and 3.
struct AxisPlan {
    int n;        // mesh cells along the axis
    int L;        // transform length (2n for y and z, n for x)
    int E;        // elements per thread (radix family: 16, 20, 24 or 36; 0: generic kernel)
    int NB;       // threads per line (0: generic kernel)
    int nst;      // number of stages
    int ntw;      // entries in the twiddle table
    int R[kMaxStages];          // radix of stage s
    int Ns[kMaxStages];         // product of the radices before stage s
    uint32_t magic[kMaxStages]; // floor(2^32 / Ns) + 1, for b / Ns
    int twoff[kMaxStages];      // offset of stage s in the twiddle table
    const void *tw;             // twiddles exp(-2 pi i r k / (Ns R)), k < Ns, 1 <= r < R
    const void *post;           // x only: exp(-i pi k / n), k < n
};

struct DevPlan {
    int nx, ny, nz, prec;  // prec: 0 = FP32, 1 = FP64
    int zb;                // z planes per tile of the workspace
    int gz;                // spectrum kz-fastest (z pass by wavefront-owned lines)
    AxisPlan ax[3];        // x, y, z
    const void *G;         // spectrum, main part
    const void *Gn;        // spectrum, kx = nx
};

// One problem inside a grouped launch.
struct ProbArg {
    const DevPlan *plan;
    const void *S;    // source (x forward pass)
    void *Phi;        // potential (x inverse pass)
    void *W;          // workspace main part
    void *Wn;         // workspace Nyquist column
};

// A run of `group` consecutive problems p[first .. first+group) with the same
// plan.  Its workgroups are numbered tile-major (tile, member), so the members
// that read the same spectrum slice are neighbours in the launch.
struct Segment {
    int wg_begin;     // first workgroup of the segment
    int first;        // index of its first problem in LaunchArgs::p
    int group;        // problems in the segment
    int wg_main;      // tiles of main lines per problem; the rest are Nyquist lines
};

// Workspace bytes of a launch above which its line data is streamed with
// nontemporal accesses: about the device's Infinity Cache (256 MB), which a
// smaller launch's workspaces can stay in between passes.
constexpr size_t kStreamBytes = size_t(256) << 20;

struct LaunchArgs {
    int count;        // problems in this launch
    int nseg;         // segments
    int nwg;          // workgroups doing work (the grid may be padded to a multiple of 8)
    int xcd_remap;    // renumber workgroups so each XCD gets a contiguous range
    int wave_z;       // z pass: spectra kz-fastest, lines kept within one wavefront
    int gtile;        // generic line kernel: lines per workgroup (a power of two)
    int glmax;        // generic line kernel: longest line of the launch
    int gtw;          // generic line kernel: stage twiddles copied into LDS after the two buffers
    int nt;           // streaming launch (workspaces beyond kStreamBytes): its line data takes
                      // nontemporal loads and stores where the kernel says so
    Segment seg[kMaxProblems];
    ProbArg p[kMaxProblems];
};

enum PassMode { X_FWD = 0, Y_FWD = 1, Z_CONV = 2, Y_INV = 3, X_INV = 4 };

// Start (in elements) of workspace row (z, ky).
__host__ __device__ inline size_t w_row(int z, int ky, int ny, int nx, int zb) {
    const int sh = __builtin_ctz(static_cast<unsigned>(zb));  // zb is a power of two
    return ((static_cast<size_t>(z >> sh) * 2 * ny + ky) * zb + (z & (zb - 1))) * static_cast<size_t>(nx);
}

// LDS layout of a workgroup (complex elements), identical on host and device.
// Column passes keep element (line c, position P) at P*col_stride + c; row passes
// at c*S + P + P/16, with S chosen so that the NB-lane chunks of consecutive
// rows fall on different banks.
__host__ __device__ constexpr int row_stride(int L, int NB, int csz) {
    int S = L + (L >> 4);
    const int chunk = NB * csz;
    if (chunk < 256) {
        const int want = chunk % 256;
        while ((S * csz) % 256 != want) ++S;
    }
    return S;
}
// Row stride (complex values) of a line in the wavefront-owned z convolution:
// the row layout's P + P/16, plus one so that the rows of neighbouring lines
// start on different banks (the tile is transposed through these rows).
__host__ __device__ constexpr int wave_line_stride(int L) { return L + L / 16 + 1; }

// Column passes: position stride of the LDS tile, tile + 1 (the extra column
// staggers the positions of a wavefront's lines over the banks), or tile where
// the LDS limits a CU to fewer than four workgroups (tile data plus the L - 1
// stage twiddles in 160 KB) and dropping that column lets one more fit:
// measured on 384-point lines, 3 workgroups per CU instead of 2 beat the bank
// staggering by 8 % per solve.
__host__ __device__ constexpr int col_stride(int L, int tile, int csz) {
    const long cap = 160 * 1024;
    const long padded = (static_cast<long>(L) * (tile + 1) + L - 1) * csz;
    const long packed = (static_cast<long>(L) * tile + L - 1) * csz;
    return cap / padded < 4 && cap / packed > cap / padded ? tile : tile + 1;
}

__host__ __device__ constexpr int data_elems(bool row, int L, int NB, int block, int csz) {
    const int tile = block / NB;
    return row ? tile * row_stride(L, NB, csz) : L * col_stride(L, tile, csz);
}

inline int pass_axis(int mode) { return mode == X_FWD || mode == X_INV ? 0 : (mode == Z_CONV ? 2 : 1); }

// Largest workgroup per (precision, radix family), chosen so that the E
// registers per thread fit without spilling.
// Default lines per workgroup: column passes take 128-byte row segments of
// complex values, row passes enough rows for 256-thread groups.
__host__ __device__ constexpr int default_tile(int prec, bool row) {
    return row ? (prec == 0 ? 32 : 16) : (prec == 0 ? 16 : 8);
}

// Lines per workgroup of pass `mode` (lines of nb threads): the default tile.
// Measured, smaller z-pass tiles (more workgroups per CU, 64- or 32-byte row
// segments) lose at every size.
__host__ __device__ constexpr int fix_tile(int prec, int mode, int /*nb*/) {
    return default_tile(prec, mode == X_FWD || mode == X_INV);
}

__host__ __device__ constexpr int max_block_for(int prec, int E) {
    return prec == 0 ? (E == 16 ? 1024 : (E <= 24 || E == 32 ? 512 : 256)) : (E == 16 ? 512 : 256);
}

// Line forms of the line-pass instances (template parameter FIX): FIX & 7 is
// the number of compile-time stages (0: run-time geometry; 2, 3 or 4: radices
// E, K / E, M, K / E, M, M, K with M the power-of-two part of E), FIX & 8 marks
// 64-bit addresses (some array of the launch reaches 4 GB; else 32-bit lane
// offsets).  fix_nb: threads per line.
__host__ __device__ constexpr int fix_stages(int fix) { return fix & 7; }
__host__ __device__ constexpr bool fix_off32(int fix) { return (fix & 7) != 0 && (fix & 8) == 0; }
__host__ __device__ constexpr int fix_nb(int fix, int E, int K) {
    return (fix & 7) == 2 ? K : ((fix & 7) == 3 ? (E & -E) * K : ((fix & 7) == 4 ? (E & -E) * (E & -E) * K : 0));
}
constexpr int kFixWide = 8;

// Lines per workgroup of a line-pass launch (pass_kernel) for lines of nb
// threads in radix family E: the default tile, halved while the workgroup
// exceeds the family's largest or its LDS (data, stage twiddles and, for rows,
// the split factors) exceeds 160 KB.  Long lines thus keep compile-time geometry
// with a smaller tile.
__host__ __device__ constexpr int pass_tile(int prec, int mode, int E, int nb) {
    const bool row = mode == X_FWD || mode == X_INV;
    const int L = E * nb, csz = prec == 0 ? 8 : 16;
    int t = default_tile(prec, row);
    if (nb <= 0) return t;  // run-time geometry
    while (t > 1) {
        const long elems = static_cast<long>(data_elems(row, L, nb, t * nb, csz)) + (L - 1) + (row ? L : 0);
        if (static_cast<long>(t) * nb <= max_block_for(prec, E) && elems * csz <= 160 * 1024) break;
        t /= 2;
    }
    return t;
}

// Row passes (X_FWD, X_INV) of compile-time lines of NB threads keep their
// stage twiddles and split factors in global memory (a table the L1 holds)
// where their pass_tile() rows alone let two workgroups share a CU and rows
// plus those 2L - 1 values let only one.
__host__ __device__ constexpr bool row_tables_global(int prec, int E, int NB) {
    const int L = E * NB, csz = prec == 0 ? 8 : 16;
    const long cap = 160 * 1024;
    const long data = static_cast<long>(data_elems(true, L, NB, pass_tile(prec, X_FWD, E, NB) * NB, csz)) * csz;
    return cap / data >= 2 && cap / (data + static_cast<long>(2 * L - 1) * csz) == 1;
}

// Column y passes (Y_FWD, Y_INV) of compile-time lines of NB threads keep their
// stage twiddles in global memory and pack the tile's positions (LDS stride =
// tile) where that lets two workgroups of pass_tile() lines share a CU and the
// layout with the twiddles in LDS lets only one.  col_ldsw: the LDS position
// stride of such a launch; col_default_lds: its bytes with the twiddles in LDS.
__host__ __device__ constexpr size_t col_default_lds(int prec, int mode, int E, int NB) {
    const int L = E * NB, csz = prec == 0 ? 8 : 16;
    const int tile = pass_tile(prec, mode, E, NB);
    return (static_cast<size_t>(L) * col_stride(L, tile, csz) + L - 1) * csz;
}
__host__ __device__ constexpr bool col_tables_global(int prec, int mode, int E, int NB) {
    if (mode != Y_FWD && mode != Y_INV) return false;
    const long L = static_cast<long>(E) * NB, csz = prec == 0 ? 8 : 16, cap = 160 * 1024;
    const long packed = L * pass_tile(prec, mode, E, NB) * csz;
    return cap / packed >= 2 && cap / static_cast<long>(col_default_lds(prec, mode, E, NB)) == 1;
}
__host__ __device__ constexpr int col_ldsw(int prec, int mode, int E, int NB) {
    const int tile = pass_tile(prec, mode, E, NB);
    return col_tables_global(prec, mode, E, NB) ? tile : col_stride(E * NB, tile, prec == 0 ? 8 : 16);
}

// Threads per line of the wavefront-owned column kernel: ST compile-time stages
// with radices E, M, K (ST = 3) or E, M, M, K (4), M = E & -E.
__host__ __device__ constexpr int wave_nb(int E, int K, int ST) {
    return ST == 4 ? (E & -E) * (E & -E) * K : (E & -E) * K;
}

// Lines per workgroup of the wavefront-owned column kernel for lines of NB
// threads, ST compile-time stages: the default tile, halved while the
// workgroup exceeds the family's largest or the tile's rows and the stage
// twiddles exceed the LDS (lines of 1536 points in the 24-family; four-stage
// lines: 1152 and 2304 points in the 36-family, 640 and 1280 in the 20-family).
__host__ __device__ constexpr int wave_tile(int prec, int mode, int E, int NB, int ST = 3) {
    int t = fix_tile(prec, mode, NB);
    const long L = static_cast<long>(E) * NB, csz = prec == 0 ? 8 : 16;
    while (t > 1 && (static_cast<long>(t) * NB > max_block_for(prec, E) ||
                     (t * static_cast<long>(wave_line_stride(static_cast<int>(L))) + L - 1) * csz > 160 * 1024))
        t /= 2;
    return t;
}

// Whether the wavefront-owned column kernel keeps the stage twiddles in LDS
// after the tile's rows: always for three-stage lines; for four-stage ones
// unless leaving them in global memory (a table the L1 holds) lets one more
// workgroup share a CU.
__host__ __device__ constexpr bool wave_tw_lds(int prec, int mode, int E, int NB, int ST = 3) {
    if (ST != 4) return true;
    const long L = static_cast<long>(E) * NB, csz = prec == 0 ? 8 : 16, cap = 160 * 1024;
    const long rows = wave_tile(prec, mode, E, NB, ST) * static_cast<long>(wave_line_stride(static_cast<int>(L))) * csz;
    return cap / rows <= cap / (rows + (L - 1) * csz);
}

// LDS bytes of the wavefront-owned column kernel of pass `mode` for lines of
// length L = E*NB: one row per line of the tile, then the stage twiddles (when
// they are kept in LDS).
__host__ __device__ constexpr size_t wave_lds_bytes(int prec, int mode, int E, int NB, int ST = 3) {
    const int L = E * NB;
    return static_cast<size_t>(wave_tile(prec, mode, E, NB, ST) * wave_line_stride(L) +
                               (wave_tw_lds(prec, mode, E, NB, ST) ? L - 1 : 0)) *
           (prec == 0 ? 8 : 16);
}

// Wavefronts per SIMD the wavefront-owned kernel is compiled for: as many as
// its workgroups that fit a CU's LDS bring (so that the register allocation
// does not keep a second workgroup out), at least one.
__host__ __device__ constexpr int wave_waves_per_simd(int prec, int mode, int E, int NB, int ST = 3) {
    if (ST != 4) return 1;
    const long per_cu = 160L * 1024 / static_cast<long>(wave_lds_bytes(prec, mode, E, NB, ST));
    const long w = per_cu * wave_tile(prec, mode, E, NB, ST) * NB / 64 / 4;
    return w < 1 ? 1 : (w > 8 ? 8 : static_cast<int>(w));
}
__host__ __device__ constexpr size_t wave_z_lds_bytes(int prec, int E, int NB) {
    return wave_lds_bytes(prec, Z_CONV, E, NB);
}

// Fused plane kernels (x and y transforms of one z plane per workgroup) for
// nx == ny = n = E*K: n*K threads, the LDS plane (n rows of row_stride(n, K))
// followed by the n - 1 stage twiddles, the n split factors and 2n values of
// column 0.
__host__ __device__ constexpr size_t plane_lds_bytes(int prec, int E, int K) {
    const int n = E * K, csz = prec == 0 ? 8 : 16;
    return static_cast<size_t>(n * row_stride(n, K, csz) + 4 * n - 1) * csz;
}
// FP64 workgroups stay at 256 threads or fewer, where the two line transforms
// each thread holds fit in registers.
__host__ __device__ constexpr bool plane_fits(int prec, int E, int K) {
    return K >= 1 && K <= (E & -E) && E * K * K <= (prec == 0 ? 1024 : 256) &&
           plane_lds_bytes(prec, E, K) <= 160 * 1024;
}

// Launchers: one per (precision, family), defined in pass_<prec>_e<E>.hip.
// K is the radix of the last stage of the pass axis (1 for a single stage).
// The plane launchers run the forward (fwd) or inverse fused kernel with n*K threads.
#define PSPFFT_DECLARE_FAMILY(NAME, PLANE)                                                          \
    hipError_t NAME(int mode, int K, int fix, const LaunchArgs &args, int grid, int block,          \
                    size_t lds, hipStream_t stream);                                                \
    hipError_t PLANE(bool fwd, int K, const LaunchArgs &args, int grid, size_t lds, hipStream_t stream);
PSPFFT_DECLARE_FAMILY(launch_f32_e16, plane_f32_e16)
PSPFFT_DECLARE_FAMILY(launch_f32_e20, plane_f32_e20)
PSPFFT_DECLARE_FAMILY(launch_f32_e24, plane_f32_e24)
PSPFFT_DECLARE_FAMILY(launch_f32_e36, plane_f32_e36)
PSPFFT_DECLARE_FAMILY(launch_f64_e16, plane_f64_e16)
PSPFFT_DECLARE_FAMILY(launch_f64_e20, plane_f64_e20)
PSPFFT_DECLARE_FAMILY(launch_f64_e24, plane_f64_e24)
PSPFFT_DECLARE_FAMILY(launch_f64_e36, plane_f64_e36)
#undef PSPFFT_DECLARE_FAMILY
// Radix family E = 32 (FP32): z lines of 2048 points (32*32*2) kept within one
// wavefront; its launcher takes only those z passes.
hipError_t launch_f32_e32(int mode, int K, int fix, const LaunchArgs &args, int grid, int block, size_t lds,
                          hipStream_t stream);

inline hipError_t launch_pass(int mode, int prec, int E, int K, int fix, const LaunchArgs &args, int grid,
                              int block, size_t lds, hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    switch (prec * 100 + E) {
        case 16: return launch_f32_e16(mode, K, fix, args, grid, block, lds, stream);
        case 20: return launch_f32_e20(mode, K, fix, args, grid, block, lds, stream);
        case 24: return launch_f32_e24(mode, K, fix, args, grid, block, lds, stream);
        case 36: return launch_f32_e36(mode, K, fix, args, grid, block, lds, stream);
        case 32: return launch_f32_e32(mode, K, fix, args, grid, block, lds, stream);
        case 116: return launch_f64_e16(mode, K, fix, args, grid, block, lds, stream);
        case 120: return launch_f64_e20(mode, K, fix, args, grid, block, lds, stream);
        case 124: return launch_f64_e24(mode, K, fix, args, grid, block, lds, stream);
        case 136: return launch_f64_e36(mode, K, fix, args, grid, block, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

inline hipError_t launch_plane(bool fwd, int prec, int E, int K, const LaunchArgs &args, int grid, size_t lds,
                               hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    switch (prec * 100 + E) {
        case 16: return plane_f32_e16(fwd, K, args, grid, lds, stream);
        case 20: return plane_f32_e20(fwd, K, args, grid, lds, stream);
        case 24: return plane_f32_e24(fwd, K, args, grid, lds, stream);
        case 36: return plane_f32_e36(fwd, K, args, grid, lds, stream);
        case 116: return plane_f64_e16(fwd, K, args, grid, lds, stream);
        case 120: return plane_f64_e20(fwd, K, args, grid, lds, stream);
        case 124: return plane_f64_e24(fwd, K, args, grid, lds, stream);
        case 136: return plane_f64_e36(fwd, K, args, grid, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

// Generic line kernel (any 2^a 3^b 5^c length): `grid` workgroups of 256
// threads, each owning args.gtile lines, with `lds` bytes of LDS (two buffers of
// gtile * (glmax + 1) complex values, then, with args.gtw, the stage twiddles).
hipError_t launch_generic(int mode, int prec, const LaunchArgs &args, int grid, size_t lds, hipStream_t stream);

// Green's-function spectrum in FP64: fills the octant (nz+1)(ny+1)(nx+1) of G
// into `a`, applies the even-extension cosine transform along each axis (using
// `b` as scratch) and writes the scaled result in plan precision into G / Gn.
// gz: store kz-fastest, G at (ky*nx + kx)*(nz+1) + kz and Gn at ky*(nz+1) + kz,
// instead of G at (kz*(ny+1) + ky)*nx + kx and Gn at kz*(ny+1) + ky.
hipError_t green_spectrum(int nx, int ny, int nz, const double h[3], int prec, int gz, double *a, double *b,
                          const double *cos_x, const double *cos_y, const double *cos_z, void *G, void *Gn,
                          hipStream_t stream);

// Copy the spectrum out as a dense (nz+1)(ny+1)(nx+1) octant, kx fastest,
// whichever layout it is kept in.
hipError_t green_export(int nx, int ny, int nz, int prec, int gz, const void *G, const void *Gn, void *dst,
                        hipStream_t stream);

}  // namespace pspfft
