// fft_core.h -- complex arithmetic and in-register DFTs for the gfx950 kernels.
// Twiddle factors inside a register DFT are compile-time constants: the compiler
// evaluates cos and sin of the rational angle 2 pi e / R in double precision and
// rounds once to the working precision.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

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
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
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

// x + b*w and x - b*w for w = exp(DIR 2 pi i e / R) with e, R known at compile
// time.  For a non-trivial w = c + i s the factor with the larger magnitude is
// taken out (Linzer and Feig's FMA butterfly): b*w = c * (b + i b tan) or
// s * (b cot + i b), so both results cost six multiply-adds instead of a full
// complex product and two additions.
template <int R, int DIR, int e, typename T>
__device__ __forceinline__ void add_sub_rot(const cx<T> x, const cx<T> b, cx<T> &sum, cx<T> &dif) {
    constexpr int em = ((e % R) + R) % R;
    if constexpr (em == 0 || 2 * em == R || 4 * em == R || 4 * em == 3 * R) {
        const cx<T> r = rot<R, DIR, e>(b);
        sum = x + r;
        dif = x - r;
    } else {
        constexpr CosSin w = turn(static_cast<long>(DIR) * em, R);
        constexpr bool eighth = 8 * em % R == 0;  // |c| = |s|: the ratio is exactly +-1
        constexpr bool cos_out = (w.c < 0 ? -w.c : w.c) >= (w.s < 0 ? -w.s : w.s);
        if constexpr (cos_out) {
            constexpr double tq = eighth ? (w.s * w.c > 0 ? 1.0 : -1.0) : w.s / w.c;
            const T t = static_cast<T>(tq), c = static_cast<T>(w.c);
            const cx<T> q = {b.x - b.y * t, b.y + b.x * t};  // b*w / c
            sum = {x.x + q.x * c, x.y + q.y * c};
            dif = {x.x - q.x * c, x.y - q.y * c};
        } else {
            constexpr double kq = w.c / w.s;
            const T k = static_cast<T>(kq), sn = static_cast<T>(w.s);
            const cx<T> q = {b.x * k - b.y, b.y * k + b.x};  // b*w / s
            sum = {x.x + q.x * sn, x.y + q.y * sn};
            dif = {x.x - q.x * sn, x.y - q.y * sn};
        }
    }
}

// Length-4 DFT of a[q] = b[q] * exp(DIR 2 pi i q k1 / R), the second layer of a
// radix-4 Cooley-Tukey split of R, with the twiddles folded into the butterflies.
template <int R, int DIR, int k1, typename T>
__device__ __forceinline__ void dft4_rot(cx<T> *b) {
    cx<T> t0, t1, t2, d;
    add_sub_rot<R, DIR, 2 * k1>(b[0], b[2], t0, t1);
    add_sub_rot<R, DIR, 3 * k1>(rot<R, DIR, k1>(b[1]), b[3], t2, d);
    const cx<T> t3 = rot<4, DIR, 1>(d);
    b[0] = t0 + t2;
    b[2] = t0 - t2;
    b[1] = t1 + t3;
    b[3] = t1 - t3;
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
                // Q = 2 and 4: the twiddles are folded into the second layer below
                if constexpr (Q == 2 || Q == 4) a[k1][q] = u[k1];
                else a[k1][q] = rot<R, DIR, q * k1>(u[k1]);
            });
        });
        sfor<0, P>([&](auto kc) {
            constexpr int k1 = decltype(kc)::value;
            if constexpr (Q == 4) {
                dft4_rot<R, DIR, k1>(a[k1]);
            } else if constexpr (Q == 2) {
                cx<T> s0, s1;
                add_sub_rot<R, DIR, k1>(a[k1][0], a[k1][1], s0, s1);
                a[k1][0] = s0;
                a[k1][1] = s1;
            } else {
                dft<Q, DIR>(a[k1]);
            }
            sfor<0, Q>([&](auto k2c) {
                constexpr int k2 = decltype(k2c)::value;
                x[k1 + P * k2] = a[k1][k2];
            });
        });
    }
}

}  // namespace pspfft
