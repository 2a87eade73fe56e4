// green.hip -- FP64 transform of the doubled Green's function, computed once
// per plan (Sec. 2.2.2: the transform of G is computed at initialisation and kept).
//
// The doubled G (Eq. greens_function) is even in every axis, so its DFT is real
// and even and equals a cosine transform of the octant 0 <= p,q,r <= n, applied
// separably along x, y and z.  The result is scaled by 1/((2nx)(2ny)(2nz)), the
// normalisation of the unnormalised forward/inverse pair, and stored in plan
// precision in the split layout of internal.h.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace pspfft {

constexpr double kPiG = 3.141592653589793238462643383279502884;

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
        v = -vol / (4.0 * kPiG * hmin);
    } else {
        const double dx = hx * p, dy = hy * q, dz = hz * r;
        v = -vol / (4.0 * kPiG * sqrt(dx * dx + dy * dy + dz * dz));
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

// Position in G (kx < nx) or Gn (kx == nx) of octant element (kx, ky, kz) whose
// dense index is i = (kz*(ny+1) + ky)*(nx+1) + kx.
__device__ __forceinline__ long green_pos(long i, int nx, int ny, int nz, int gz, bool &nyq) {
    const long kx = i % (nx + 1);
    const long row = i / (nx + 1);  // kz*(ny+1) + ky
    nyq = kx == nx;
    if (!gz) return nyq ? row : row * nx + kx;
    const long kz = row / (ny + 1), ky = row - kz * (ny + 1);
    return nyq ? ky * (nz + 1) + kz : (ky * nx + kx) * (nz + 1) + kz;
}

template <typename T>
__global__ void green_store(const double *a, int nx, int ny, int nz, int gz, double s, T *G, T *Gn) {
    const long total = static_cast<long>(nx + 1) * (ny + 1) * (nz + 1);
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    bool nyq;
    const long q = green_pos(i, nx, ny, nz, gz, nyq);
    const T v = static_cast<T>(a[i] * s);
    if (nyq) Gn[q] = v;
    else G[q] = v;
}

template <typename T>
__global__ void green_load(const T *G, const T *Gn, int nx, int ny, int nz, int gz, T *dst) {
    const long total = static_cast<long>(nx + 1) * (ny + 1) * (nz + 1);
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    bool nyq;
    const long q = green_pos(i, nx, ny, nz, gz, nyq);
    dst[i] = nyq ? Gn[q] : G[q];
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

hipError_t green_spectrum(int nx, int ny, int nz, const double h[3], int prec, int gz, double *a, double *b,
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
        hipLaunchKernelGGL(green_store<float>, dim3(nb), dim3(256), 0, stream, b, nx, ny, nz, gz, s,
                           static_cast<float *>(G), static_cast<float *>(Gn));
    else
        hipLaunchKernelGGL(green_store<double>, dim3(nb), dim3(256), 0, stream, b, nx, ny, nz, gz, s,
                           static_cast<double *>(G), static_cast<double *>(Gn));
    return hipGetLastError();
}

hipError_t green_export(int nx, int ny, int nz, int prec, int gz, const void *G, const void *Gn, void *dst,
                        hipStream_t stream) {
    const long total = static_cast<long>(nx + 1) * (ny + 1) * (nz + 1);
    const unsigned nb = static_cast<unsigned>((total + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(green_load<float>, dim3(nb), dim3(256), 0, stream, static_cast<const float *>(G),
                           static_cast<const float *>(Gn), nx, ny, nz, gz, static_cast<float *>(dst));
    else
        hipLaunchKernelGGL(green_load<double>, dim3(nb), dim3(256), 0, stream, static_cast<const double *>(G),
                           static_cast<const double *>(Gn), nx, ny, nz, gz, static_cast<double *>(dst));
    return hipGetLastError();
}

}  // namespace pspfft
