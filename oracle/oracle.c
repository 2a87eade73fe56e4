/*
 * oracle.c -- plain, slow, FP64 CPU reference for the isolated Poisson solve of
 * Budiardja & Cardall, "Parallel FFT-based Poisson Solver for Isolated
 * Three-dimensional Systems" (arXiv:1106.0557), Sec. 2.1.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls this
 * file; only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no code, header, table or constant with the HIP path.
 *
 * What it computes (all in double precision):
 *   - oracle_dft_1d     textbook O(L^2) discrete Fourier transform.
 *   - oracle_fft_1d     naive recursive mixed-radix (any prime factor) FFT,
 *                       decimation in time, no blocking or reordering tricks.
 *   - oracle_fft_axis   1D transforms along one axis of a 3D array.
 *   - oracle_fft_3d     3D transform as three sets of 1D transforms (Sec. 2.2.2).
 *   - oracle_green_value     the discrete Green's function, Eq. (greens2) at
 *                            integer index offsets, with the self-cell value of
 *                            Eq. (greens_function).
 *   - oracle_green_doubled   the Green's function on the doubled mesh, set up with
 *                            the explicit reflection rules of Eq. (greens_function).
 *   - oracle_green_hat_octant  transform of the doubled Green's function, octant
 *                            k in [0,n] per axis, divided by (2nx)(2ny)(2nz).
 *   - oracle_solve_fft  Hockney's mesh-doubling convolution (Sec. 2.1, Fig. 1):
 *                       zero-pad S, transform S and G, multiply, inverse
 *                       transform, normalise AFTER the inverse, extract the
 *                       active octant.
 *   - oracle_direct     the aperiodic discrete convolution written out as a
 *                       direct sum over all source cells (Eq. (convolution)
 *                       with Eq. (greens2) as midpoint quadrature), with
 *                       Neumaier-compensated summation.
 *
 * Array conventions: real 3D arrays are [nz][ny][nx] with x fastest; complex
 * arrays are interleaved (re, im) doubles with the same ordering.
 * Transform sign convention: forward uses exp(-2 pi i j k / L), inverse
 * exp(+2 pi i j k / L), both unnormalised.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------- 1D DFT -- */

/* Textbook definition: out[k] = sum_j in[j] exp(sign 2 pi i j k / L). */
void oracle_dft_1d(int L, const double *in, double *out, int sign) {
    for (int k = 0; k < L; ++k) {
        cplx acc = 0;
        for (int j = 0; j < L; ++j) {
            long m = ((long)j * k) % L;
            double ang = sign * 2.0 * M_PI * (double)m / (double)L;
            acc += (in[2 * j] + I * in[2 * j + 1]) * (cos(ang) + I * sin(ang));
        }
        out[2 * k] = creal(acc);
        out[2 * k + 1] = cimag(acc);
    }
}

static int smallest_factor(int n) {
    for (int p = 2; (long)p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/*
 * y[k] = sum_{j<n} x[j*stride] w^{(N/n) j k}, where w[j] = exp(sign 2 pi i j/N)
 * is the root table of the top-level length N.  Decimation in time on the
 * smallest prime factor p of n: X[k + m q] = sum_r w_n^{r (k + m q)} Y_r[k],
 * with Y_r the length-m transform of the r-th decimated subsequence.
 */
static void fft_rec(int n, const cplx *x, long stride, cplx *y, const cplx *w, int N) {
    if (n == 1) {
        y[0] = x[0];
        return;
    }
    int p = smallest_factor(n), m = n / p;
    for (int r = 0; r < p; ++r) fft_rec(m, x + r * stride, stride * p, y + (long)r * m, w, N);
    long s = N / n;
    cplx t[p];
    for (int k = 0; k < m; ++k) {
        for (int r = 0; r < p; ++r) t[r] = y[(long)r * m + k];
        for (int q = 0; q < p; ++q) {
            cplx acc = 0;
            for (int r = 0; r < p; ++r) acc += w[(((long)r * (k + (long)m * q)) % n) * s] * t[r];
            y[k + (long)m * q] = acc;
        }
    }
}

static cplx *root_table(int N, int sign) {
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    for (int j = 0; j < N; ++j) {
        double ang = sign * 2.0 * M_PI * (double)j / (double)N;
        w[j] = cos(ang) + I * sin(ang);
    }
    return w;
}

void oracle_fft_1d(int L, const double *in, double *out, int sign) {
    cplx *w = root_table(L, sign);
    cplx *x = (cplx *)malloc(sizeof(cplx) * (size_t)L);
    cplx *y = (cplx *)malloc(sizeof(cplx) * (size_t)L);
    for (int j = 0; j < L; ++j) x[j] = in[2 * j] + I * in[2 * j + 1];
    fft_rec(L, x, 1, y, w, L);
    for (int j = 0; j < L; ++j) {
        out[2 * j] = creal(y[j]);
        out[2 * j + 1] = cimag(y[j]);
    }
    free(w);
    free(x);
    free(y);
}

/* In-place transform of one axis of a complex [nz][ny][nx] array. */
static void fft_axis(cplx *a, int nx, int ny, int nz, int axis, int sign) {
    int L = axis == 0 ? nx : axis == 1 ? ny : nz;
    long estride = axis == 0 ? 1 : axis == 1 ? nx : (long)nx * ny;
    long nlines = (long)nx * ny * nz / L;
    cplx *w = root_table(L, sign);
#pragma omp parallel
    {
        cplx *x = (cplx *)malloc(sizeof(cplx) * (size_t)L);
        cplx *y = (cplx *)malloc(sizeof(cplx) * (size_t)L);
#pragma omp for schedule(static)
        for (long line = 0; line < nlines; ++line) {
            long base;
            if (axis == 0) {
                base = line * nx;
            } else if (axis == 1) {
                long z = line / nx, xx = line % nx;
                base = z * (long)nx * ny + xx;
            } else {
                base = line; /* line enumerates (y, x) of one plane */
            }
            for (int j = 0; j < L; ++j) x[j] = a[base + j * estride];
            fft_rec(L, x, 1, y, w, L);
            for (int j = 0; j < L; ++j) a[base + j * estride] = y[j];
        }
        free(x);
        free(y);
    }
    free(w);
}

/* In-place transform of one axis (0 = x, 1 = y, 2 = z) of a complex [nz][ny][nx] array. */
void oracle_fft_axis(int nx, int ny, int nz, double *a, int axis, int sign) {
    fft_axis((cplx *)a, nx, ny, nz, axis, sign);
}

void oracle_fft_3d(int nx, int ny, int nz, double *a, int sign) {
    cplx *c = (cplx *)a;
    fft_axis(c, nx, ny, nz, 0, sign);
    fft_axis(c, nx, ny, nz, 1, sign);
    fft_axis(c, nx, ny, nz, 2, sign);
}

/* ------------------------------------------------------ Green's function -- */

/*
 * Eq. (greens2) at integer offsets (p,q,r) != 0:
 *     G = - hx hy hz / (4 pi sqrt(hx^2 p^2 + hy^2 q^2 + hz^2 r^2)),
 * and the self-cell value of Eq. (greens_function):
 *     G(0,0,0) = - hx hy hz / (4 pi min(hx,hy,hz)).
 */
double oracle_green_value(long p, long q, long r, const double h[3]) {
    double vol = h[0] * h[1] * h[2];
    if (p == 0 && q == 0 && r == 0) {
        double hmin = h[0];
        if (h[1] < hmin) hmin = h[1];
        if (h[2] < hmin) hmin = h[2];
        return -vol / (4.0 * M_PI * hmin);
    }
    double d2 = h[0] * h[0] * (double)(p * p) + h[1] * h[1] * (double)(q * q) +
                h[2] * h[2] * (double)(r * r);
    return -vol / (4.0 * M_PI * sqrt(d2));
}

/*
 * Doubled-mesh Green's function g[(k*2ny + j)*2nx + i], i < 2nx etc., built by
 * the reflection rules of Eq. (greens_function): for 0 <= p,q,r <= n the value
 * G_{p,q,r} is written to (p,q,r) and to all seven mirror images obtained by
 * replacing an index p by 2n - p (taken modulo 2n, so that p = 0 maps to itself).
 */
void oracle_green_doubled(int nx, int ny, int nz, const double h[3], double *g) {
    long Nx = 2L * nx, Ny = 2L * ny, Nz = 2L * nz;
    for (long r = 0; r <= nz; ++r)
        for (long q = 0; q <= ny; ++q)
            for (long p = 0; p <= nx; ++p) {
                double v = oracle_green_value(p, q, r, h);
                long ps[2] = {p % Nx, (Nx - p) % Nx};
                long qs[2] = {q % Ny, (Ny - q) % Ny};
                long rs[2] = {r % Nz, (Nz - r) % Nz};
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c) g[(rs[c] * Ny + qs[b]) * Nx + ps[a]] = v;
            }
}

/*
 * Transform of the doubled Green's function, kept on the octant
 * 0 <= kx <= nx, 0 <= ky <= ny, 0 <= kz <= nz and divided by (2nx)(2ny)(2nz):
 * out[(kz*(ny+1) + ky)*(nx+1) + kx] = Re(G~(k)) / (8 nx ny nz).
 * Returns (scaled) max |Im G~| over the whole doubled mesh in *imag_max and
 * max |G~| in *abs_max.
 */
void oracle_green_hat_octant(int nx, int ny, int nz, const double h[3], double *out,
                             double *imag_max, double *abs_max) {
    long Nx = 2L * nx, Ny = 2L * ny, Nz = 2L * nz, N = Nx * Ny * Nz;
    double *g = (double *)malloc(sizeof(double) * (size_t)N);
    double *a = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    oracle_green_doubled(nx, ny, nz, h, g);
    for (long i = 0; i < N; ++i) {
        a[2 * i] = g[i];
        a[2 * i + 1] = 0.0;
    }
    free(g);
    oracle_fft_3d((int)Nx, (int)Ny, (int)Nz, a, -1);
    double scale = 1.0 / (double)N, im = 0.0, ab = 0.0;
    for (long i = 0; i < N; ++i) {
        double ai = fabs(a[2 * i + 1]) * scale, aa = hypot(a[2 * i], a[2 * i + 1]) * scale;
        if (ai > im) im = ai;
        if (aa > ab) ab = aa;
    }
    for (long kz = 0; kz <= nz; ++kz)
        for (long ky = 0; ky <= ny; ++ky)
            for (long kx = 0; kx <= nx; ++kx)
                out[(kz * (ny + 1) + ky) * (nx + 1) + kx] = a[2 * ((kz * Ny + ky) * Nx + kx)] * scale;
    if (imag_max) *imag_max = im;
    if (abs_max) *abs_max = ab;
    free(a);
}

/* ------------------------------------------------------ the solve itself -- */

/*
 * Hockney mesh doubling (Sec. 2.1): S on the active octant, zero elsewhere;
 * Phi = IDFT(DFT(S) * DFT(G)) / ((2nx)(2ny)(2nz)) on the active octant.
 * Returns 0 on success, -1 on allocation failure.
 */
int oracle_solve_fft(int nx, int ny, int nz, const double h[3], const double *S, double *Phi) {
    long Nx = 2L * nx, Ny = 2L * ny, Nz = 2L * nz, N = Nx * Ny * Nz;
    double *g = (double *)malloc(sizeof(double) * (size_t)N);
    double *a = (double *)calloc(2 * (size_t)N, sizeof(double));
    double *b = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    if (!g || !a || !b) {
        free(g);
        free(a);
        free(b);
        return -1;
    }
    oracle_green_doubled(nx, ny, nz, h, g);
    for (long i = 0; i < N; ++i) {
        b[2 * i] = g[i];
        b[2 * i + 1] = 0.0;
    }
    free(g);
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) a[2 * ((z * Ny + y) * Nx + x)] = S[(z * ny + y) * nx + x];
    oracle_fft_3d((int)Nx, (int)Ny, (int)Nz, a, -1);
    oracle_fft_3d((int)Nx, (int)Ny, (int)Nz, b, -1);
    cplx *ca = (cplx *)a, *cb = (cplx *)b;
    for (long i = 0; i < N; ++i) ca[i] *= cb[i];
    free(b);
    oracle_fft_3d((int)Nx, (int)Ny, (int)Nz, a, +1);
    double scale = 1.0 / (double)N;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x)
                Phi[(z * ny + y) * nx + x] = a[2 * ((z * Ny + y) * Nx + x)] * scale;
    free(a);
    return 0;
}

/*
 * Direct aperiodic sum, Phi_t = sum_{s in active} G(t - s) S_s, at the flat
 * target indices targets[0..ntargets) (index = (z*ny + y)*nx + x).  G depends on
 * |dx|,|dy|,|dz| only, so it is tabulated once on [0,nz)x[0,ny)x[0,nx).
 * Neumaier (compensated) summation keeps the sum accurate to ~1 ulp.
 */
int oracle_direct(int nx, int ny, int nz, const double h[3], const double *S, long ntargets,
                  const long *targets, double *out) {
    long nxy = (long)nx * ny, n = nxy * nz;
    double *tab = (double *)malloc(sizeof(double) * (size_t)n);
    if (!tab) return -1;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < nz; ++r)
        for (long q = 0; q < ny; ++q)
            for (long p = 0; p < nx; ++p) tab[(r * ny + q) * nx + p] = oracle_green_value(p, q, r, h);
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < ntargets; ++t) {
        long ti = targets[t];
        long tz = ti / nxy, ty = (ti / nx) % ny, tx = ti % nx;
        double sum = 0.0, comp = 0.0;
        for (long z = 0; z < nz; ++z) {
            long dz = labs(tz - z);
            for (long y = 0; y < ny; ++y) {
                long dy = labs(ty - y);
                const double *srow = S + (z * ny + y) * nx;
                const double *grow = tab + (dz * ny + dy) * nx;
                for (long x = 0; x < nx; ++x) {
                    double term = grow[labs(tx - x)] * srow[x];
                    double tsum = sum + term;
                    if (fabs(sum) >= fabs(term))
                        comp += (sum - tsum) + term;
                    else
                        comp += (term - tsum) + sum;
                    sum = tsum;
                }
            }
        }
        out[t] = sum + comp;
    }
    free(tab);
    return 0;
}
