// internal.h -- data structures shared by the HIP kernels and the host runtime.
//
// Workspace layout of one in-flight solve (complex values of the precision):
//   W  : [z < nz][ky < 2ny][kx < nx]   main part, row stride nx (rows aligned)
//   Wn : [z < nz][ky < 2ny]            the kx = nx (Nyquist) column, split off so
//                                      that every row of W has an aligned length
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

// One line length L = 2n along one axis, split into stages of radix R[s].
// A line is handled by NB = L / E threads, each owning the E positions
// t + NB*m (m < E) before the first and after the last stage.
struct AxisPlan {
    int n;        // mesh cells along the axis
    int L;        // transform length, 2n
    int E;        // elements per thread (radix family: 16, 20, 24 or 36)
    int NB;       // threads per line
    int nst;      // number of stages
    int pad_;
    int R[kMaxStages];          // radix of stage s
    int Ns[kMaxStages];         // product of the radices before stage s
    uint32_t magic[kMaxStages]; // floor(2^32 / Ns) + 1, for b / Ns
    int twoff[kMaxStages];      // offset of stage s in the twiddle table
    const void *tw;             // twiddles exp(-2 pi i r k / (Ns R)), k < Ns, 1 <= r < R
};

struct DevPlan {
    int nx, ny, nz, prec;  // prec: 0 = FP32, 1 = FP64
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
    int wg_begin;     // first workgroup of this problem in the launch
    int wg_main;      // workgroups for the main lines; the rest handle Nyquist lines
};

struct LaunchArgs {
    int count;        // problems in this launch
    int pad_;
    ProbArg p[kMaxProblems];
};

enum PassMode { X_FWD = 0, Y_FWD = 1, Z_CONV = 2, Y_INV = 3, X_INV = 4 };

inline int pass_axis(int mode) { return mode == X_FWD || mode == X_INV ? 0 : (mode == Z_CONV ? 2 : 1); }

// Launchers (defined in pspfft_kernels.hip).  `block` threads per workgroup,
// `lds_bytes` dynamic shared memory.
hipError_t launch_pass(int mode, int prec, int E, const LaunchArgs &args, int grid, int block,
                       size_t lds_bytes, hipStream_t stream);
int max_block(int prec, int E);

// Green's-function spectrum in FP64: fills the octant (nz+1)(ny+1)(nx+1) of G
// into `a`, applies the even-extension cosine transform along each axis (using
// `b` as scratch) and writes the scaled result in plan precision into G / Gn.
hipError_t green_spectrum(int nx, int ny, int nz, const double h[3], int prec, double *a, double *b,
                          const double *cos_x, const double *cos_y, const double *cos_z, void *G, void *Gn,
                          hipStream_t stream);

// Copy the spectrum out as a dense (nz+1)(ny+1)(nx+1) octant.
hipError_t green_export(int nx, int ny, int nz, int prec, const void *G, const void *Gn, void *dst,
                        hipStream_t stream);

}  // namespace pspfft
