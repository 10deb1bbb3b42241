// Device-side definitions of libsphjet (gfx950, wave64).
//
// Data layout on the device (structure of arrays, one slot per particle, slots
// ordered by (cell key, particle id) after every sort):
//   pos   double2   FP64 positions (exact pair predicate, no drift at 1e-4 dx)
//   vel   V2<T>     velocity
//   dens  T         rho - rho0 (keeps the Tait pressure accurate in FP32)
//   mass  T
//   tag   uint32    (system << 4) | type
//   id    uint32    caller's particle id
//   cell  uint32    global cell key of the slot (system base + cx * ny + cy)
// Cell keys put the y index fastest, so the (2R+1) x (2R+1) block of cells
// around a particle is 2R+1 contiguous slot ranges, one per cell row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sphjet {

enum : uint32_t { T_FLUID = 0, T_WALL = 1, T_PISTON = 2, T_INACTIVE = 3 };
// Instability bits of the flags word, and one informational bit: a half step
// in which some particle moved farther than half the cell skin, so its
// evaluation scanned the cells again instead of walking the skin mask.
enum : uint32_t { FLAG_NONFINITE = 1, FLAG_DENSITY = 2, FLAG_SKIN = 4, FLAG_RESCAN = 8 };

// Largest cell reach of such a rescan: a particle that moved farther than
// (RESCAN_MAX_REACH s - 2h)/2 in half a step raises FLAG_SKIN.
constexpr int RESCAN_MAX_REACH = 6;

template <typename T> struct V2t;
template <> struct V2t<float> { using type = float2; };
template <> struct V2t<double> { using type = double2; };
template <typename T> using V2 = typename V2t<T>::type;
template <typename T> struct V4t;
template <> struct V4t<float> { using type = float4; };
template <> struct V4t<double> { using type = double4; };
template <typename T> using V4 = typename V4t<T>::type;

// The colour sweep records which of a particle's candidates passed the pair
// predicate as one 32-bit word per cell row of its block (at most 5 rows): bit
// k of word r is the k-th slot of row r's slot range. Row 4 keeps bits 0..30;
// bit 31 of word 4 marks a particle with a row of more candidates than its
// word holds, whose later sweeps scan its cells again instead.
constexpr uint32_t MASK_ROW_BITS = 32;
constexpr uint32_t MASK_OVERFLOW = 1u << 31;

// The mask words of one particle.
struct RowMask {
    uint32_t w[5];
};

// Per-system constants, precomputed on the host.
template <typename T>
struct SysDev {
    // neighbour grid (FP64, so keys and the predicate are exact)
    double x0, y0, inv_s, R2;      // grid origin, 1/cell size, (2h)^2
    double skin2;                  // (half the skin)^2: allowed half-step displacement squared
    double cell_s;                 // cell size s
    double Rs2;                    // (R s)^2: radius^2 of the skin mask kept for the half step
    int32_t nx, ny, reach, kernel;
    uint32_t cell_base, pad_;
    float r2_in, r2_out;           // FP32 band around (2h)^2 outside which FP32 decides the predicate
    // physics in the working precision
    T h, inv_h, wnorm, gnorm;      // W = wnorm * w(q); grad_a W = gnorm * g(q) * r_ab
    T W0;                          // W(0)
    T rho0, inv_rho0, B, c0;       // Tait: P = B((1 + delta)^gamma - 1), delta = dens / rho0
    T gamma, half_gm1;             // gamma, (gamma - 1)/2
    T alpha_h, eta2;               // alpha * h, eta^2
    T visc_c0;                     // -alpha h c0: c_b scaled for the viscosity term (gamma = 7)
    T sigma, eps;                  // surface tension, eps = eps_h / h
    T gx, gy;
    int32_t gamma7, closure;
    T closure_tol;
    int32_t density_sum;           // 1: eq. 6 for fluid particles
    int32_t boundary;              // 1: repulsive-force walls (eq. 29)
    int32_t g_plane, pad2_;        // 1: g acts only where r . g_hat >= g_from
    double ghx, ghy, g_from;
    double h64, wnorm64, rho0_64;  // FP64 copies for the density summation
    // time stepping (FP64)
    double courant, dt_fixed;
    double box_lo_x, box_lo_y, box_hi_x, box_hi_y;
    double pdx, pdy, pu, pamp, pomega;
};

__device__ __forceinline__ uint32_t tag_type(uint32_t t) { return t & 15u; }
__device__ __forceinline__ uint32_t tag_sys(uint32_t t) { return t >> 4; }

// Cell coordinate of x on an axis with origin lo and ncell cells; out-of-range
// (and NaN) values clamp to the edge cells. No FMA: the key must be bit-exact.
__device__ __forceinline__ int cell_coord(double x, double lo, double inv, int ncell) {
#pragma clang fp contract(off)
    double t = floor((x - lo) * inv);
    if (!(t >= 0.0)) t = 0.0;
    double top = (double)(ncell - 1);
    if (t > top) t = top;
    return (int)t;
}

// Exact FP64 pair predicate pieces: r_ab = r_a - r_b and |r_ab|^2 without FMA.
__device__ __forceinline__ double pair_r2(double2 pa, double2 pb, double& dx, double& dy) {
#pragma clang fp contract(off)
    dx = pa.x - pb.x;
    dy = pa.y - pb.y;
    return dx * dx + dy * dy;
}

// The same predicate |r_ab|^2 < (2h)^2, decided mostly in FP32. fx, fy are
// the FP64 components ex, ey rounded to FP32 and r2f = fx^2 + fy^2 in FP32
// (contracted or not): each component carries one rounding, each square and
// the sum one more, so r2f is within 2^-21 of the FP64 |r_ab|^2 (itself within
// 2^-52 of the exact value). r2_in and r2_out sit 2^-19 of (2h)^2 either side
// of it, so below r2_in (above r2_out) the FP64 verdict is certainly "inside"
// ("outside"); in the band between, the FP64 sum decides, formed as above.
// The band is so thin (a few in 10^6 of the candidates) that the FP64 branch
// is almost never taken by any lane of a wave.
__device__ __forceinline__ bool pair_within(double ex, double ey, float r2f, float r2_in, float r2_out, double R2) {
    if (r2f < r2_in) return true;
    if (__builtin_expect(r2f > r2_out, 1)) return false;
    double fx, fy;
    return pair_r2(make_double2(ex, ey), make_double2(0.0, 0.0), fx, fy) < R2;
}

// Element i of a particle array through a 32-bit byte offset (the particle
// count is limited so that every array's byte offsets fit): the loads then take
// the array's base from scalar registers and one 32-bit offset per lane.
template <typename U>
__device__ __forceinline__ const U& at(const U* base, uint32_t i) {
    return *reinterpret_cast<const U*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(U));
}

template <typename T> __device__ __forceinline__ T rcp(T x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }

template <typename T> __device__ __forceinline__ T sqrt_(T x);
template <> __device__ __forceinline__ float sqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double sqrt_<double>(double x) { return __builtin_sqrt(x); }

// Constants of a system's smoothing kernel, loaded once per thread.
template <typename T>
struct KernelConsts {
    int kernel;
    T inv_h, wnorm, gnorm;
};

template <typename T>
__device__ __forceinline__ KernelConsts<T> kconsts(const SysDev<T>& S) {
    return KernelConsts<T>{S.kernel, S.inv_h, S.wnorm, S.gnorm};
}

// Kernel value and gradient factor at distance r (< 2h): W(r) and F(r) with
// grad_a W_ab = F(r) r_ab.
//   Wendland: W = wn (1 - q/2)^4 (1 + 2q),  F = -5 wn / h^2 (1 - q/2)^3
//   cubic:    W = wn [1 - 1.5 q^2 + 0.75 q^3 | 0.25 (2 - q)^3],
//             F = wn / h^2 [-3 + 2.25 q | -0.75 (2 - q)^2 / q]
template <typename T>
__device__ __forceinline__ void kernel_wf(const KernelConsts<T>& K, T r, T& W, T& F) {
    T q = r * K.inv_h;
    if (K.kernel == 0) {
        T u = T(1) - T(0.5) * q;
        T u3 = u * u * u;
        W = K.wnorm * u3 * u * (T(1) + T(2) * q);
        F = K.gnorm * u3;
    } else {
        if (q <= T(1)) {
            W = K.wnorm * (T(1) + q * q * (T(-1.5) + T(0.75) * q));
            F = K.gnorm * (T(-3) + T(2.25) * q);
        } else {
            T u = T(2) - q;
            W = K.wnorm * T(0.25) * u * u * u;
            F = K.gnorm * T(-0.75) * u * u * rcp(q);
        }
    }
}

// W(r) / wnorm: the kernel's shape, for sums that apply the normalisation once.
template <typename T>
__device__ __forceinline__ T kernel_shape(const KernelConsts<T>& K, T r) {
    T q = r * K.inv_h;
    if (K.kernel == 0) {
        T u = T(1) - T(0.5) * q;
        T u2 = u * u;
        return u2 * u2 * (T(1) + T(2) * q);
    }
    if (q <= T(1)) return T(1) + q * q * (T(-1.5) + T(0.75) * q);
    T u = T(2) - q;
    return T(0.25) * u * u * u;
}

// W / wnorm in FP64, at q = r / h (the density summation's terms).
__device__ __forceinline__ double kernel_shape64(int kernel, double q) {
    if (kernel == 0) {
        const double u = 1.0 - 0.5 * q;
        const double u2 = u * u;
        return u2 * u2 * (1.0 + 2.0 * q);
    }
    if (q <= 1.0) return 1.0 + q * q * (-1.5 + 0.75 * q);
    const double u = 2.0 - q;
    return 0.25 * u * u * u;
}

template <typename T>
__device__ __forceinline__ T kernel_f(const KernelConsts<T>& K, T r) {
    T q = r * K.inv_h;
    if (K.kernel == 0) {
        T u = T(1) - T(0.5) * q;
        return K.gnorm * u * u * u;
    }
    if (q <= T(1)) return K.gnorm * (T(-3) + T(2.25) * q);
    T u = T(2) - q;
    return K.gnorm * T(-0.75) * u * u * rcp(q);
}

// Tait equation: P / rho^2 from the stored deviation dens = rho - rho0. With
// gamma = 7, (1 + d)^7 - 1 is expanded in d so a small compression keeps its
// relative precision.
template <typename T>
__device__ __forceinline__ void tait(const SysDev<T>& S, T dens, T& rho, T& p_over_rho2) {
    T d = dens * S.inv_rho0;
    rho = S.rho0 + dens;
    T irho = rcp(rho);
    T P;
    if (S.gamma7) {
        T e = d * (T(7) + d * (T(21) + d * (T(35) + d * (T(35) + d * (T(21) + d * (T(7) + d))))));
        P = S.B * e;
    } else {
        P = S.B * expm1(S.gamma * log1p(d));
    }
    p_over_rho2 = P * irho * irho;
}

// Sound speed of the Tait equation, c = c0 (rho / rho0)^((gamma - 1) / 2),
// from the density itself (the sweeps keep rho, not c, per particle).
template <typename T>
__device__ __forceinline__ T sound_speed(const SysDev<T>& S, T rho) {
    const T s = rho * S.inv_rho0;
    if (S.gamma7) return S.c0 * s * s * s;
    return S.c0 * exp(S.half_gm1 * log(s));
}

// -alpha h c(rho): the sound speed as the viscosity term (eq. 10) uses it.
template <typename T>
__device__ __forceinline__ T visc_speed(const SysDev<T>& S, T rho) {
    const T s = rho * S.inv_rho0;
    if (S.gamma7) return S.visc_c0 * s * s * s;
    return -S.alpha_h * S.c0 * exp(S.half_gm1 * log(s));
}

// m / rho, which the colour sum needs of every neighbour.
template <typename T>
__device__ __forceinline__ T particle_vol(const SysDev<T>& S, T dens, T mass) {
    return mass * rcp(S.rho0 + dens);
}

template <typename T>
__device__ __forceinline__ T tait_pressure(const SysDev<T>& S, T dens) {
    T rho, pr;
    tait(S, dens, rho, pr);
    return pr * rho * rho;
}

// Whether gravity acts on a fluid particle at pa (everywhere, or beyond a plane
// normal to g: r . g_hat >= g_from, formed without FMA as the oracle forms it).
template <typename T>
__device__ __forceinline__ bool gravity_on(const SysDev<T>& S, double2 pa) {
#pragma clang fp contract(off)
    return !S.g_plane || pa.x * S.ghx + pa.y * S.ghy >= S.g_from;
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Maximum of non-negative values over the wave: the unsigned maximum of the
// bit patterns (the same order for non-negative numbers), one shuffle and one
// integer max per step.
__device__ __forceinline__ float wave_max_nonneg(float x) {
    uint32_t u = __float_as_uint(x);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) u = max(u, (uint32_t)__shfl_xor((int)u, o, 64));
    return __uint_as_float(u);
}
__device__ __forceinline__ double wave_max_nonneg(double x) {
    unsigned long long u = (unsigned long long)__double_as_longlong(x);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long q = __shfl_xor(u, o, 64);
        u = q > u ? q : u;
    }
    return __longlong_as_double((long long)u);
}

// atomicMin on the bit pattern of a non-negative double, skipped when the
// stored value is already no larger (values only decrease between the clears,
// so a stale read can only cost an unneeded atomic): thousands of waves
// update one minimum per system, and most of them cannot lower it.
__device__ __forceinline__ void atomic_min_bits(unsigned long long* dst, double m) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
    const unsigned long long cur = __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bits < cur) atomicMin(dst, bits);
}

// Minimum of non-negative values v into dst[sys] (stored as FP64 bits, whose
// unsigned order equals the numeric order for non-negative numbers). Every lane
// of the wave must call this (from uniform control flow); lanes with valid =
// false contribute nothing. The wave is taken one system at a time: a wave
// minimum and one atomic per distinct system among its lanes.
__device__ __forceinline__ void atomic_min_per_system(unsigned long long* dst, int stride, int sys,
                                                      double v, bool valid) {
    const bool live = valid && v < __builtin_inf();
    unsigned long long todo = __ballot(live);
    while (todo) {
        const int l = __ffsll((long long)todo) - 1;
        const int s0 = __builtin_amdgcn_readfirstlane(__shfl(sys, l, 64));
        const bool mine = live && sys == s0;
        const double m = wave_min(mine ? v : __builtin_inf());
        if (__lane_id() == 0) atomic_min_bits(dst + (size_t)s0 * stride, m);
        todo &= ~__ballot(mine);
    }
}

// Workgroup id remapped so that the workgroups one XCD receives (hardware
// dispatches them round-robin over the 8 XCDs) cover one contiguous range of
// slots: neighbouring tiles then share that XCD's L2.
__device__ __forceinline__ int tile_index(int xcd_remap) {
    int g = (int)gridDim.x, i = (int)blockIdx.x;
    if (!xcd_remap) return i;
    int q = g >> 3, r = g & 7, x = i & 7, k = i >> 3;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace sphjet
