// pibm_device.h -- gfx950 kernels of the coupled thermal LBM-PIBM-DEM step.
//
// Zhang, Yuan, Trias, Yu, Tan & Oliva, arXiv 1502.01159:
//   Sec. 2.1  BGK for f (Eq. lbm2) and g (Eq. lbm2.5), equilibria (lbm3,
//             lbm3.5), macroscopic moments with half-force / half-source;
//   Sec. 2.2  PIBM: Lagrange interpolation (lbm5-lbm6), point exchange
//             (lbm7, lbm7.5, lbm8), Guo forcing (lbm9), spreading with the
//             cosine kernel (lbm10-lbm12), heat source (lbm12.5, lbm12.6),
//             reaction on the particle (lbm13);
//   Sec. 2.3  DEM: Newton-Euler (demgov), Hertz normal and
//             Mindlin-Deresiewicz tangential contact.
//
// Data layout in HBM: structure of arrays, population q of node n at
// q * Ns + n, n = (k * ny + j) * nx + i (x fastest), two copies (A read,
// B written) swapped every step.  Populations are stored as deviations from
// the rest state, f - w (rho0 = 1) and g - w T_s; 16-bit storage keeps the
// deviation divided by w so that every direction uses the same range, with
// T_s the middle of the case's initial temperatures (T_s = T_ref otherwise).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <type_traits>

namespace pibm {

// --------------------------------------------------------------------------
// Lattices.  Flow: D2Q9 / D3Q19 BGK, or the D3Q15 of Sec. 2.1.  Temperature:
// D2Q5 / D3Q7 with a linear equilibrium, c_sg^2 = 1/3 (D2Q5) and 1/4 (D3Q7).
// --------------------------------------------------------------------------
template <int DIM, int QF> struct LatT;

template <> struct LatT<2, 9> {
    static constexpr int Q = 9, QG = 5;
    __host__ __device__ static constexpr int e(int q, int d) {
        // rest, +x, +y, -x, -y, (+x+y), (-x+y), (-x-y), (+x-y)
        return d == 2 ? 0
             : d == 0 ? (q == 1 || q == 5 || q == 8 ? 1 : (q == 3 || q == 6 || q == 7 ? -1 : 0))
                      : (q == 2 || q == 5 || q == 6 ? 1 : (q == 4 || q == 7 || q == 8 ? -1 : 0));
    }
    __host__ __device__ static constexpr int opp(int q) {
        return q == 0 ? 0 : q == 1 ? 3 : q == 2 ? 4 : q == 3 ? 1 : q == 4 ? 2 : q == 5 ? 7 : q == 6 ? 8 : q == 7 ? 5 : 6;
    }
    __host__ __device__ static constexpr double w(int q) { return q == 0 ? 4.0 / 9.0 : (q < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
    __host__ __device__ static constexpr double wg(int q) { return q == 0 ? 1.0 / 3.0 : 1.0 / 6.0; }
    static constexpr double csg2_inv = 3.0;
    static constexpr bool QT = false;      // thermal equilibrium linear in u
};

template <> struct LatT<3, 19> {
    static constexpr int Q = 19, QG = 7;
    // rest; +-x, +-y, +-z; then the 12 edge directions in opposite pairs
    __host__ __device__ static constexpr int e(int q, int d) {
        return d == 0 ? (q == 1 || q == 7 || q == 9 || q == 11 || q == 13 ? 1
                         : (q == 2 || q == 8 || q == 10 || q == 12 || q == 14 ? -1 : 0))
             : d == 1 ? (q == 3 || q == 7 || q == 10 || q == 15 || q == 17 ? 1
                         : (q == 4 || q == 8 || q == 9 || q == 16 || q == 18 ? -1 : 0))
                      : (q == 5 || q == 11 || q == 14 || q == 15 || q == 18 ? 1
                         : (q == 6 || q == 12 || q == 13 || q == 16 || q == 17 ? -1 : 0));
    }
    __host__ __device__ static constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
    __host__ __device__ static constexpr double w(int q) { return q == 0 ? 1.0 / 3.0 : (q < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
    __host__ __device__ static constexpr double wg(int q) { return q == 0 ? 0.25 : 0.125; }
    static constexpr double csg2_inv = 4.0;
    static constexpr bool QT = false;
};

// D3Q15 (Sec. 2.1): rest; +-x, +-y, +-z; then the 8 corners in opposite pairs
// (+,+,+) (-,-,-) (+,+,-) (-,-,+) (+,-,+) (-,+,-) (-,+,+) (+,-,-);
// w = 2/9, 1/9, 1/72.  Same thermal lattice (D3Q7).
template <> struct LatT<3, 15> {
    static constexpr int Q = 15, QG = 7;
    __host__ __device__ static constexpr int e(int q, int d) {
        return q == 0 ? 0
             : q < 7 ? ((q - 1) / 2 == d ? ((q & 1) ? 1 : -1) : 0)
                     : (d == 0 ? (q == 7 || q == 9 || q == 11 || q == 14 ? 1 : -1)
                        : d == 1 ? (q == 7 || q == 9 || q == 12 || q == 13 ? 1 : -1)
                                 : (q == 7 || q == 10 || q == 11 || q == 13 ? 1 : -1));
    }
    __host__ __device__ static constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
    __host__ __device__ static constexpr double w(int q) { return q == 0 ? 2.0 / 9.0 : (q < 7 ? 1.0 / 9.0 : 1.0 / 72.0); }
    __host__ __device__ static constexpr double wg(int q) { return q == 0 ? 0.25 : 0.125; }
    static constexpr double csg2_inv = 4.0;
    static constexpr bool QT = false;
};

template <int DIM> using Lat = LatT<DIM, DIM == 2 ? 9 : 19>;

// Lattice facts checked at compile time: opposite directions, unit weight
// sum, second moment c_s^2 = 1/3 and isotropic fourth moment (1/9 for xxyy,
// 1/3 for xxxx).
template <class L> constexpr bool lattice_ok()
{
    double w0 = 0, wxx = 0, wxy = 0, wxxyy = 0, wxxxx = 0;
    for (int q = 0; q < L::Q; ++q) {
        for (int d = 0; d < 3; ++d)
            if (L::e(L::opp(q), d) != -L::e(q, d)) return false;
        const double ex = L::e(q, 0), ey = L::e(q, 1);
        w0 += L::w(q); wxx += L::w(q) * ex * ex; wxy += L::w(q) * ex * ey;
        wxxyy += L::w(q) * ex * ex * ey * ey; wxxxx += L::w(q) * ex * ex * ex * ex;
    }
    auto near = [](double a, double b) { return a - b < 1e-15 && b - a < 1e-15; };
    return near(w0, 1.0) && near(wxx, 1.0 / 3.0) && near(wxy, 0.0) && near(wxxyy, 1.0 / 9.0) && near(wxxxx, 1.0 / 3.0);
}
static_assert(lattice_ok<LatT<2, 9>>(), "D2Q9 table");
static_assert(lattice_ok<LatT<3, 19>>(), "D3Q19 table");
static_assert(lattice_ok<LatT<3, 15>>(), "D3Q15 table");

// Temperature on the flow lattice itself, with the flow's quadratic
// equilibrium form (Sec. 2.1 as printed): every flow direction, the flow
// weights, c_sg^2 = 1/3.
template <class L> struct SameThermal : L {
    static constexpr int QG = L::Q;
    __host__ __device__ static constexpr double wg(int q) { return L::w(q); }
    static constexpr double csg2_inv = 3.0;
    static constexpr bool QT = true;
};

// The lattices of a kernel instance travel with its storage traits: a traits
// class with QF = 15 selects D3Q15 for the flow, one with QTH = 1 the
// temperature on the flow lattice; otherwise the defaults.
template <class Base> struct OnQ15 : Base { static constexpr int QF = 15; };
template <class Base> struct OnQuadT : Base { static constexpr int QTH = 1; };
template <class SF, class = void> struct FlowQ { static constexpr int value = 0; };
template <class SF> struct FlowQ<SF, decltype((void)SF::QF)> { static constexpr int value = SF::QF; };
template <class SF, class = void> struct ThermQ { static constexpr int value = 0; };
template <class SF> struct ThermQ<SF, decltype((void)SF::QTH)> { static constexpr int value = SF::QTH; };
template <int DIM, class SF>
using FlowLatOf = LatT<DIM, DIM == 3 && FlowQ<SF>::value == 15 ? 15 : (DIM == 2 ? 9 : 19)>;
template <int DIM, class SF>
using LatOf = typename std::conditional<ThermQ<SF>::value == 1, SameThermal<FlowLatOf<DIM, SF>>, FlowLatOf<DIM, SF>>::type;

// --------------------------------------------------------------------------
// Counter-based uniform numbers for stochastic rounding: a 32-bit integer
// hash (xorshift-multiply finaliser) of (node, population, step).
// --------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16; x *= 0x7feb352du;
    x ^= x >> 15; x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
// Sixteen random bits per stored value, in the top half of the returned
// word: one hash per node and step, and an odd multiple of it per value (the
// high or the low half of the product, the latter rotated up: a shift would
// be folded into the multiply, which then runs at quarter rate).
__device__ __forceinline__ uint32_t node_seed(uint32_t n, uint32_t step_seed)
{
    return mix32(n * 0x9e3779b1u ^ step_seed);
}
__device__ __forceinline__ uint32_t sr_bits(uint32_t seed, int k)
{
    // 24-bit product (full-rate multiply) of the seed with an odd constant
    const uint32_t P = __umul24(seed, ((uint32_t)(2 * (k >> 1) + 1) * 0x9e3779b1u) & 0xffffffu);
    return (k & 1) ? __builtin_amdgcn_alignbit(P, P, 16) : P;
}

// --------------------------------------------------------------------------
// Storage traits: decode a stored deviation to T; store old + increment.
// FP32 and the 16-bit formats round the store stochastically: random bits
// are added below the kept mantissa and the rest is cut off, which rounds
// the magnitude up with probability equal to the cut-off fraction (to 2^-16
// of an ulp).  Increments smaller than half an ulp of a slowly changing
// population are so kept on average instead of being discarded every step;
// the hash makes it reproducible bit for bit.  `w` is the lattice weight of
// the direction (16-bit formats store dev / w).
// The lattice update's stores are non-temporal: the next copy is read only
// in the next step, and keeping it out of L2 leaves room there for the
// neighbouring tiles' rows that this step's gathers read again.
// --------------------------------------------------------------------------
struct SpreadF48; struct SpreadF32; struct SpreadD64;
struct StF32 {
    using S = float; using T = float; using C = double;
    using Spread = SpreadF48;
    static constexpr bool SCALED = false;     // stored deviation is f - w (not divided by w)
    static __device__ __forceinline__ T cvt(S v, double) { return v; }
    static __device__ __forceinline__ void st(S *p, T v, double) { *p = v; }
    static __device__ __forceinline__ void st_sum(S *p, T old, C inc, double, uint32_t rnd)
    {
        // double -> float keeps 24 of 53 mantissa bits: randomise the top 16
        // of the 29 cut
        unsigned long long b = (unsigned long long)__double_as_longlong((double)old + inc);
        b = (b + ((unsigned long long)(rnd >> 16) << 13)) & ~0x1fffffffull;
        __builtin_nontemporal_store((float)__longlong_as_double((long long)b), p);
    }
};
struct StF64 {
    using S = double; using T = double; using C = double;
    using Spread = SpreadD64;
    static constexpr bool SCALED = false;
    static __device__ __forceinline__ T cvt(S v, double) { return v; }
    static __device__ __forceinline__ void st(S *p, T v, double) { *p = v; }
    static __device__ __forceinline__ void st_sum(S *p, T old, C inc, double, uint32_t)
    {
        __builtin_nontemporal_store(old + inc, p);
    }
};
typedef __attribute__((ext_vector_type(2))) _Float16 h2x;   // the conversions' packed results
typedef __attribute__((ext_vector_type(2))) __bf16 bf2x;
struct StF16 {
    using S = __half; using T = float; using C = float;
    using Spread = SpreadF48;
    static constexpr bool SCALED = true;      // stored deviation is (f - w) / w
    static __device__ __forceinline__ T cvt(S v, double w) { return __half2float(v) * (float)w; }
    static __device__ __forceinline__ void st(S *p, T v, double w) { *p = __float2half_rn(v * (float)(1.0 / w)); }
    static __device__ __forceinline__ void st_sum(S *p, T old, C inc, double w, uint32_t rnd)
    {
        // gfx950's stochastic-rounding conversion: the top 13 bits of rnd are
        // added below the half's 11 significant bits and the rest is cut
        // (subnormal halves likewise; NaN and infinity kept)
        const float s = (old + inc) * (float)(1.0 / w);
        const h2x v = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(h2x, rnd), s, rnd, false);   // high half unused
        __builtin_nontemporal_store((unsigned short)(__builtin_bit_cast(uint32_t, v) & 0xffffu), (unsigned short *)p);
    }
};
struct StBF16 {
    using S = uint16_t; using T = float; using C = float;
    using Spread = SpreadF32;
    static constexpr bool SCALED = true;
    static __device__ __forceinline__ T cvt(S v, double w) { return __uint_as_float(((uint32_t)v) << 16) * (float)w; }
    static __device__ __forceinline__ void st(S *p, T v, double w)
    {
        const uint32_t u = __float_as_uint(v * (float)(1.0 / w));
        // round to nearest even; NaN stays NaN
        const uint32_t r = (u & 0x7fffffffu) > 0x7f800000u ? (u | 0x00400000u) : u + 0x7fffu + ((u >> 16) & 1u);
        *p = (uint16_t)(r >> 16);
    }
    static __device__ __forceinline__ void st_sum(S *p, T old, C inc, double w, uint32_t rnd)
    {
        // stochastic-rounding conversion: the top 16 bits of rnd are added
        // below the kept 8 significant bits and the rest is cut
        const float s = (old + inc) * (float)(1.0 / w);
        const bf2x v = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(bf2x, rnd), s, rnd, false);
        __builtin_nontemporal_store((uint16_t)(__builtin_bit_cast(uint32_t, v) & 0xffffu), p);
    }
};


// --------------------------------------------------------------------------
// Shared records.
// --------------------------------------------------------------------------
struct DevParticle {               // 128 bytes, FP64
    double x[3], u[3], om[3], th[3];
    double R, rho_r, T;
    int flags, tmpl;
};
struct DevReact {                  // per-particle reactions of the last step
    double F[3], tq[3], H, dTA;
};
// A point record: 64 bytes with FP32 values (half a 128-byte line, never
// straddling two) and 96 with FP64.  The cosine-kernel weights of one axis
// pair up: delta(-1-t) + delta(1-t) = delta(-t) + delta(2-t) = 1/2 (Eq.
// lbm12), so the record keeps those of nodes b-1 and b, and nodes b+1 and b+2
// take 1/2 minus them (each axis's four weights sum to 1 by construction).
template <typename T> struct alignas(sizeof(T) == 4 ? 64 : 32) MarkerRec {
    int b[3];                      // floor(X_l) per axis (unwrapped)
    int pad;
    T w[3][2];                     // cosine-kernel weights of nodes b-1 and b per axis
    T fa[3];                       // F_l A_l (force density times weight)
    T qa;                          // Q_l A_l
};
static_assert(sizeof(MarkerRec<float>) == 64 && sizeof(MarkerRec<double>) == 96, "point record sizes");

enum : int {
    ERR_FIELD = 1,        // NaN / out-of-range rho or |u|
    ERR_CONTACTS = 2,     // contact slots exhausted
    ERR_NEIGHBOURS = 4,   // neighbour list full
    ERR_STALE = 8,        // a particle moved more than skin/2 since the list was built
    ERR_DOMAIN = 16,      // particle centre outside the walls / NaN state
    ERR_TILES = 32,       // tile lists full
};

// Once the watchdog word is set the state is no longer meaningful; every
// kernel of the following steps returns at entry (the host reports the error
// at its next synchronisation).  Kernels with barriers take the decision once
// per workgroup so that all of its threads agree.
__device__ __forceinline__ bool halted(const int *err) { return __atomic_load_n(err, __ATOMIC_RELAXED) != 0; }

__device__ __forceinline__ bool block_halted(const int *err)
{
    __shared__ int s_halt;
    if (threadIdx.x == 0) s_halt = halted(err) ? 1 : 0;
    __syncthreads();
    return s_halt != 0;
}

// A particle centre that can be turned into lattice indices: finite and
// within 1e8 of the origin.  Kernels that derive indices from a centre flag
// any other state (ERR_DOMAIN) and skip the particle instead of converting
// it: a float-to-int conversion of NaN or of a runaway value is undefined.
__device__ __forceinline__ bool centre_ok(const DevParticle &P, int dim)
{
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok = ok && (d >= dim || fabs(P.x[d]) < 1.0e8);   // constant indices
    return ok;
}

constexpr int TILE_X = 64;
template <int DIM> struct Tile {
    static constexpr int X = TILE_X, Y = DIM == 3 ? 4 : 16, Z = DIM == 3 ? 4 : 1;
    static constexpr int N = X * Y * Z;           // 1024 nodes, 4 per thread
    // LDS layout of the tile's spread force: rows padded to 68 words so that
    // a marker footprint (4 x 4 x 4 nodes, one per lane) lands on 64
    // distinct banks: offset = x + 68 y + 272 z = x + 4 y + 16 z (mod 64).
    static constexpr int PY = X + 4, PZ = PY * Y;
    static constexpr int NPAD = PZ * Z;
    static __host__ __device__ constexpr int lds(int x, int y, int z) { return x + PY * y + PZ * z; }
};
constexpr int LBM_THREADS = 256;

template <typename T> struct LbmArgs {
    int nx, ny, nz;
    int per[3];
    long long Ns;                  // stride between population arrays (elements)
    int ntx, nty, ntz, ntiles;
    double omf, omg;               // 1 / tau
    double gf, gg;                 // 1 - 1 / (2 tau)
    double gbeta;
    double Tref;                   // the g deviations are stored from w Tref (T_ref, or for 16-bit storage the
                                   // middle of the case's initial temperatures)
    double dTb;                    // Tref - T_ref: buoyancy acts on T - T_ref = (T - Tref) + dTb
    double tw[6];                  // T_wall - Tref per face
    const void *fA, *gA;
    void *fB, *gB;
    const int *tile_start, *tile_count;
    const int2 *tile_items;        // items: a particle patch's first point record and its point count
    const MarkerRec<T> *mk;
    int *err;
    T *macro;                      // macro pass: rho, u[3], T at k * Ns + n
    uint32_t step;                 // step counter
    uint32_t seed;                 // hash of the step counter (stochastic-rounding stream)
};

// --------------------------------------------------------------------------
// Neighbour coordinates of a node (wrap on periodic axes, invalid at walls).
// --------------------------------------------------------------------------
struct Nbr {
    int m[3], p[3];                // coordinate - 1, + 1
    bool vm[3], vp[3];
};

__device__ __forceinline__ void nbr_axis(int c, int n, int per, int &m, int &p, bool &vm, bool &vp)
{
    m = c - 1; p = c + 1; vm = true; vp = true;
    if (c == 0) { if (per) m = n - 1; else vm = false; }
    if (c == n - 1) { if (per) p = 0; else vp = false; }
}

// Pull streaming (Eqs. lbm2, lbm2.5 read at the arrival node): deviation
// populations of node (x, y, z) after streaming, with halfway bounce-back for
// f and anti-bounce-back (Dirichlet wall temperature) for g.  Branch-free:
// every direction loads from one selected address (the upstream node in its
// own array, or this node in the opposite direction's array at a wall), so
// all loads of a node are in flight together.  Addresses are 32-bit byte
// offsets from the first array of the direction's opposite pair (a
// wave-uniform base), which the host bounds below 4 GiB.
template <class S>
__device__ __forceinline__ S load_at(const S *base, uint32_t elem)
{
    return *(const S *)((const char *)base + (uint32_t)(elem * (uint32_t)sizeof(S)));
}
template <class S>
__device__ __forceinline__ S *addr_at(S *base, uint32_t elem)
{
    return (S *)((char *)base + (uint32_t)(elem * (uint32_t)sizeof(S)));
}

// RAW (lattice kernel, storage that divides the deviation by w): the values
// are returned as stored, still divided by w, and the anti-bounce-back
// Dirichlet value is divided by w too (w_q = w of the opposite direction).
template <int DIM, class SF, class T, class TG, bool RAW = false>
__device__ __forceinline__ void pull(const LbmArgs<T> &a, int x, int y, int z, T *f, TG *g)
{
    using L = LatOf<DIM, SF>;
    using S = typename SF::S;
    const S *fa = (const S *)a.fA;
    const S *ga = (const S *)a.gA;
    Nbr nb;
    nbr_axis(x, a.nx, a.per[0], nb.m[0], nb.p[0], nb.vm[0], nb.vp[0]);
    nbr_axis(y, a.ny, a.per[1], nb.m[1], nb.p[1], nb.vm[1], nb.vp[1]);
    if (DIM == 3) nbr_axis(z, a.nz, a.per[2], nb.m[2], nb.p[2], nb.vm[2], nb.vp[2]);
    else { nb.m[2] = nb.p[2] = 0; nb.vm[2] = nb.vp[2] = true; }
    const uint32_t nx = (uint32_t)a.nx, sxy = (uint32_t)a.nx * (uint32_t)a.ny, Ns = (uint32_t)a.Ns;
    // element offsets of the upstream coordinate per axis: index by e + 1
    const uint32_t ox[3] = {(uint32_t)nb.p[0], (uint32_t)x, (uint32_t)nb.m[0]};
    const uint32_t oy[3] = {(uint32_t)nb.p[1] * nx, (uint32_t)y * nx, (uint32_t)nb.m[1] * nx};
    const uint32_t oz[3] = {(uint32_t)nb.p[2] * sxy, (uint32_t)z * sxy, (uint32_t)nb.m[2] * sxy};
    const bool vx[3] = {nb.vp[0], true, nb.vm[0]};
    const bool vy[3] = {nb.vp[1], true, nb.vm[1]};
    const bool vz[3] = {nb.vp[2], true, nb.vm[2]};
    const uint32_t self = oz[1] + oy[1] + ox[1];
    S fr[L::Q], gr[L::QG];
    bool gv[L::QG];
    int gface[L::QG];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const int ex = L::e(q, 0) + 1, ey = L::e(q, 1) + 1, ez = L::e(q, 2) + 1;
        const int o = L::opp(q), lo = q < o ? q : o;
        const bool v = vx[ex] && vy[ey] && vz[ez];
        const uint32_t off = v ? (uint32_t)(q - lo) * Ns + (oz[ez] + oy[ey] + ox[ex]) : (uint32_t)(o - lo) * Ns + self;
        fr[q] = load_at(fa + (size_t)lo * a.Ns, off);
    }
#pragma unroll
    for (int q = 0; q < L::QG; ++q) {
        const int ex = L::e(q, 0) + 1, ey = L::e(q, 1) + 1, ez = L::e(q, 2) + 1;
        const int o = L::opp(q), lo = q < o ? q : o;
        gv[q] = vx[ex] && vy[ey] && vz[ez];
        // the wall that blocks the direction (the last blocked axis when a
        // diagonal meets an edge) sets the Dirichlet temperature
        gface[q] = !vz[ez] ? 4 + (ez == 2 ? 0 : 1) : (!vy[ey] ? 2 + (ey == 2 ? 0 : 1) : (ex == 2 ? 0 : 1));
        const uint32_t off = gv[q] ? (uint32_t)(q - lo) * Ns + (oz[ez] + oy[ey] + ox[ex]) : (uint32_t)(o - lo) * Ns + self;
        gr[q] = load_at(ga + (size_t)lo * a.Ns, off);
    }
    // every load of the node is issued before any value is used
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) f[q] = SF::cvt(fr[q], RAW ? 1.0 : L::w(q));
#pragma unroll
    for (int q = 0; q < L::QG; ++q) {
        const TG val = (TG)SF::cvt(gr[q], RAW ? 1.0 : L::wg(q));
        g[q] = gv[q] ? val : -val + (TG)(2.0 * (RAW ? 1.0 : L::wg(q)) * a.tw[gface[q]]);
    }
}

// Raw moments of the streamed deviations: rho - 1, j, S - T_s (T_s: the g storage offset, Tref).
template <int DIM, class L, class C, class T>
__device__ __forceinline__ void moments(const T *f, const C *g, C &drho, C *j, C &dS)
{
    drho = 0; j[0] = 0; j[1] = 0; j[2] = 0; dS = 0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        drho += f[q];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            if (L::e(q, d) > 0) j[d] += f[q];
            else if (L::e(q, d) < 0) j[d] -= f[q];
        }
    }
#pragma unroll
    for (int q = 0; q < L::QG; ++q) dS += g[q];
}

// --------------------------------------------------------------------------
// Cosine kernel weights of Eq. (lbm12) for the four nodes b-1 .. b+2 around a
// point at b + t, 0 <= t < 1: with c = cos(pi t / 2), s = sin(pi t / 2),
//   delta(-1-t) = (1 - s)/4, delta(-t) = (1 + c)/4,
//   delta(1-t)  = (1 + s)/4, delta(2-t) = (1 - c)/4.
// --------------------------------------------------------------------------
__device__ __forceinline__ void cos_weights(float t, float *w)
{
    float s, c;
    sincospif(0.5f * t, &s, &c);
    w[0] = 0.25f * (1.0f - s); w[1] = 0.25f * (1.0f + c); w[2] = 0.25f * (1.0f + s); w[3] = 0.25f * (1.0f - c);
}
__device__ __forceinline__ void cos_weights(double t, double *w)
{
    double s, c;
    sincospi(0.5 * t, &s, &c);
    w[0] = 0.25 * (1.0 - s); w[1] = 0.25 * (1.0 + c); w[2] = 0.25 * (1.0 + s); w[3] = 0.25 * (1.0 - c);
}

__device__ __forceinline__ int wrap_or_out(int c, int n, int per)
{
    if (per) { c %= n; if (c < 0) c += n; return c; }
    return (c < 0 || c >= n) ? -1 : c;
}


// --------------------------------------------------------------------------
// K1: fused pull-stream + moments + PIBM spreading (Eqs. lbm10-lbm12,
// lbm12.6) + buoyancy + Guo-forced BGK for f (lbm2, lbm3, lbm9) and
// source-forced BGK for g (lbm2.5, lbm12.5).  One workgroup per 1024-node
// tile; nothing of the spreading is written to HBM.
//
// Spreading in three steps per wave: (1) each lane tests one Lagrangian
// point of the tile's particle list against the tile and counts the rows
// (fixed y, z) of its 4^d footprint that lie in the tile; (2) a wave prefix
// sum appends one (point, row) entry per such row to the wave's LDS queue;
// (3) whenever 64 entries are queued, each lane takes one and adds the
// row's four nodes into the tile's accumulators.  The accumulators are
// integer fixed point (the Spread formats below): integer addition does not depend on order,
// so the result is the same bit for bit whatever the interleaving of lanes,
// waves and list entries, with no atomics on floating point.
// --------------------------------------------------------------------------
// Fixed-point format of the spreading accumulators, per storage format.
// A contribution is a component v of a point record (clamped to |v| <= LIM,
// which also maps NaN to a finite value that the node's velocity check then
// flags) times the SCALE and one kernel weight w per axis.
// FP32 storage (FP32 records): resolution 2^-36.  term() forms v w + 1.5 2^52
// in one FP64 FMA; the product of the two floats is exact, and the sum's low
// 48 bits hold round(v w) in two's complement on top of the shifter's bits,
// which lie above bit 47.  The accumulator adds these words unchanged: the
// shifters pile up above bit 47 only, so the low 48 bits, sign-extended once
// per node, are the exact sum while it stays below 2^47 (|F_B|, |Q_B| < 2048
// at a node; a maximal contribution is 2^41, and any state the watchdog lets
// run is orders of magnitude below).
// BF16 storage (FP32 records): 32-bit accumulators at 2^-24, from the low
// 32 bits of the same FMA; exact while |F_B|, |Q_B| < 128 at a node (a
// maximal contribution, |v| = 32, is 2^26).  They halve the tile's LDS (22.8
// instead of 39.4 KB), so that a fifth workgroup fits on a CU.  A typical
// contribution (a point force near 1e-4 times a kernel weight of a few
// hundredths) is a few tens of units, so each is rounded by a percent or
// more: still below what BF16's own rounding (2^-9) puts in the fields; FP16
// storage keeps the 48-bit format, since at this resolution its velocity
// error grew threefold.

// FP64 storage (FP64 records, the parity path): resolution 2^-50, |v| <= 64,
// exact round-to-nearest conversion, int64 sums.
struct SpreadF48 {
    using A = unsigned long long;
    static constexpr float SCALE = 0x1p36f, LIM = 256.0f;
    static __device__ __forceinline__ A term(double v, double w)
    {
        return (A)__double_as_longlong(fma(v, w, 0x1.8p52));
    }
    static __device__ __forceinline__ double value(A a) { return (double)((long long)(a << 16) >> 16) * 0x1p-36; }
};
struct SpreadF32 {
    using A = unsigned int;
    static constexpr float SCALE = 0x1p24f, LIM = 32.0f;
    static __device__ __forceinline__ A term(double v, double w)
    {
        return (A)(unsigned long long)__double_as_longlong(fma(v, w, 0x1.8p52));
    }
    static __device__ __forceinline__ double value(A a) { return (double)(int)a * 0x1p-24; }
};
struct SpreadD64 {
    using A = unsigned long long;
    static constexpr double SCALE = 0x1p50, LIM = 64.0;
    static __device__ __forceinline__ A term(double v, double w) { return (A)(long long)rint(v * w); }
    static __device__ __forceinline__ double value(A a) { return (double)(long long)a * 0x1p-50; }
};

// Node index on one axis: wrapped on periodic axes, unchanged otherwise (a
// node outside the domain never lies in a tile's interior range, or lies in
// a ragged tile's padding, which the node phase skips).
__device__ __forceinline__ int spread_axis(int c, int n, int per)
{
    if (per) { c %= n; if (c < 0) c += n; }
    return c;
}
// Exclusive prefix sum over the wave of cnt (0 <= cnt < 2^BITS) and the total.
template <int BITS>
__device__ __forceinline__ int wave_prefix(int cnt, int &total)
{
    int pre = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < BITS; ++bit) {
        const unsigned long long bm = __ballot((cnt >> bit) & 1);
        pre += (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bm, 0u)) << bit;
        tot += __popcll(bm) << bit;
    }
    total = tot;
    return pre;
}


constexpr int XCD_CHUNK = 8;
constexpr int TILE_STREAMS = 2;
__device__ __forceinline__ int xcd_tile(int b, int G)
{
    const int span = 8 * XCD_CHUNK;
    const int main = G - G % span;
    if (b >= main) return b;
    const int xcd = b & 7, slot = b >> 3;
    // Groups of `span` consecutive tiles are dispatched from TILE_STREAMS
    // contiguous parts of the domain in turn, each part in its own order:
    // particles fill some regions only (the top third in sedimentation), and
    // this keeps the workgroups that spread points beside ones that only
    // stream, instead of leaving all spreading to one stretch of the launch.
    const int NG = main / span, r = slot / XCD_CHUNK;
    const int per = NG / TILE_STREAMS, extra = NG % TILE_STREAMS;
    int part, i;
    if (r < per * TILE_STREAMS) { part = r % TILE_STREAMS; i = r / TILE_STREAMS; }
    else { part = r - per * TILE_STREAMS; i = per; }            // the longer parts' last groups
    const int g = part * per + min(part, extra) + i;
    return g * span + xcd * XCD_CHUNK + slot % XCD_CHUNK;
}

template <int DIM, class SF, bool MACRO>
__global__ __launch_bounds__(LBM_THREADS) void k_lbm(LbmArgs<typename SF::T> a)
{
    using T = typename SF::T;
    using L = LatOf<DIM, SF>;
    using TL = Tile<DIM>;
    constexpr int NC = DIM + 1;
    // A point's footprint has 4 rows (fixed y) per z layer; each append
    // queues the rows of one z layer (2D: its only layer), at most 4 per lane,
    // and follows a drain to below 128 entries.  The small queue keeps the
    // workgroup's LDS under 40 KB: four workgroups per CU.
    constexpr int RMAX = 4;                           // rows appended per lane at a time
    constexpr int QCAP = 128 + 64 * RMAX;            // < 128 queued before each append
    constexpr int KSCAN = 4;                          // chunks whose loads are in flight together
    // fixed-point F_B, Q_B per tile node; rows (fixed y, z) padded to X + 1
    // words so that the rows of one point's footprint, queued on adjacent
    // lanes, fall on different LDS banks
    constexpr int PXU = TL::X + 1, NROW = TL::Y * TL::Z;
    using SP = typename SF::Spread;
    __shared__ typename SP::A acc[NC][NROW * PXU];
    __shared__ int queue[LBM_THREADS / 64][QCAP];

    // XCD-aware order: consecutive workgroups go to different XCDs (round
    // robin over 8); give each XCD runs of XCD_CHUNK consecutive tiles so that
    // x-neighbours share an L2, while the runs interleave over the domain so
    // that regions dense in particles are spread over all XCDs.
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = t % a.ntx, rem = t / a.ntx, ty = rem % a.nty, tz = rem / a.nty;
    const int x0 = tx * TL::X, y0 = ty * TL::Y, z0 = tz * TL::Z;
    const int tid = threadIdx.x;
    if (block_halted(a.err)) return;

    const int ps = a.tile_start[t], pe = ps + a.tile_count[t];
    const bool has = pe > ps;
    if (has) {
        const int lane = tid & 63, wv = tid >> 6;
        // the first 64 entries of the tile's list of particle patches, loaded
        // while the accumulators are cleared
        int pm0 = 0, pn = 0;
        if (lane < pe - ps) {
            const int2 it = a.tile_items[ps + lane];
            pm0 = it.x;
            pn = it.y;
        }
        for (int i = tid; i < NC * NROW * PXU; i += LBM_THREADS) (&acc[0][0])[i] = 0;
        __syncthreads();
        int *q = queue[wv];
        int qn = 0;                                   // wave-uniform queue length

        // (3) a queued (point, row) entry: the row's nodes x = b-1 .. b+2.
        // fetch() only issues the loads, so that two batches are in flight
        // together; apply() adds the contributions.
        struct Row { int4 b; T w[3][2]; T f[NC]; int ky, kz; };
        auto fetch = [&](int code, Row &r) {
            const int m = code >> 4;
            r.ky = (code >> 2) & 3;
            r.kz = code & 3;
            const MarkerRec<T> *R = a.mk + m;
            r.b = *(const int4 *)&R->b[0];
#pragma unroll
            for (int d = 0; d < DIM; ++d) { r.w[d][0] = R->w[d][0]; r.w[d][1] = R->w[d][1]; }
#pragma unroll
            for (int c = 0; c < NC; ++c) r.f[c] = c < DIM ? R->fa[c] : R->qa;
        };
        auto apply = [&](const Row &r) {
            const int ly = spread_axis(r.b.y - 1 + r.ky, a.ny, a.per[1]) - y0;
            const int lz = DIM == 3 ? spread_axis(r.b.z - 1 + r.kz, a.nz, a.per[2]) - z0 : 0;
            const int row = PXU * (ly + TL::Y * lz);
            // the axis weights of nodes b-1 .. b+2: w0, w1, 1/2 - w0, 1/2 - w1
            const T wa = r.w[0][0], wb = r.w[0][1];
            const T w0[4] = {wa, wb, (T)0.5 - wa, (T)0.5 - wb};
            const T yk = (r.ky & 1) ? r.w[1][1] : r.w[1][0];
            const T wy = r.ky < 2 ? yk : (T)0.5 - yk;
            T wz = (T)1;
            if (DIM == 3) {
                const T zk = (r.kz & 1) ? r.w[2][1] : r.w[2][0];
                wz = r.kz < 2 ? zk : (T)0.5 - zk;
            }
            const T wyz = wy * wz;
            double v[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T cl = fmin(fmax(r.f[c], (T)-SP::LIM), (T)SP::LIM);   // NaN -> -limit
                v[c] = (double)(cl * (T)SP::SCALE * wyz);
            }
#pragma unroll
            for (int kx = 0; kx < 4; ++kx) {
                const int lx = spread_axis(r.b.x - 1 + kx, a.nx, a.per[0]) - x0;
                if (lx >= 0 && lx < TL::X) {
                    const double wx = (double)w0[kx];
#pragma unroll
                    for (int c = 0; c < NC; ++c) atomicAdd(&acc[c][row + lx], SP::term(v[c], wx));
                }
            }
        };
        auto drain2 = [&](int ca, bool va, int cb, bool vb) {
            Row ra, rb;
            if (va) fetch(ca, ra);
            if (vb) fetch(cb, rb);
            if (va) apply(ra);
            if (vb) apply(rb);
        };
        // (1) + (2) for one point (m < 0: none) with base cell b
        auto scan = [&](int m, int4 b) {
            int cnt = 0, ymask = 0, zmask = 1;
            if (m >= 0) {
                bool xin = false;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int lx = spread_axis(b.x - 1 + k, a.nx, a.per[0]) - x0;
                    xin = xin || (lx >= 0 && lx < TL::X);
                    const int ly = spread_axis(b.y - 1 + k, a.ny, a.per[1]) - y0;
                    ymask |= (ly >= 0 && ly < TL::Y) ? (1 << k) : 0;
                }
                if (DIM == 3) {
                    zmask = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int lz = spread_axis(b.z - 1 + k, a.nz, a.per[2]) - z0;
                        zmask |= (lz >= 0 && lz < TL::Z) ? (1 << k) : 0;
                    }
                }
                cnt = xin ? __popc(ymask) : 0;        // rows per z layer
            }
            // not unrolled: the drain below would be copied 16-fold into the scan's 4 unrolled calls
#pragma unroll 1
            for (int kz = 0; kz < (DIM == 3 ? 4 : 1); ++kz) {
                const int c = ((zmask >> kz) & 1) ? cnt : 0;
                int tot;
                int pos = qn + wave_prefix<3>(c, tot);
                if (c) {
#pragma unroll
                    for (int ky = 0; ky < 4; ++ky)
                        if ((ymask >> ky) & 1) q[pos++] = (m << 4) | (ky << 2) | kz;
                }
                qn += tot;
                __builtin_amdgcn_wave_barrier();
                while (qn >= 128) {
                    qn -= 128;
                    const int ca = q[qn + lane], cb = q[qn + 64 + lane];
                    __builtin_amdgcn_wave_barrier();
                    drain2(ca, true, cb, true);
                }
            }
        };

        // The list in batches of 64 patches; within a batch the points of
        // all its patches form one virtual array, cut into chunks of 64
        // that the waves take in turn (chunk0 carries the turn across
        // batches), KSCAN chunks per wave at a time.
        int chunk0 = 0;
        for (int e0 = ps; e0 < pe; e0 += 64) {
            const int ne = min(64, pe - e0);
            if (e0 != ps) {
                pm0 = 0; pn = 0;
                if (lane < ne) {
                    const int2 it = a.tile_items[e0 + lane];
                    pm0 = it.x;
                    pn = it.y;
                }
            }
            int incl = pn;                            // inclusive prefix over the batch
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int y = __shfl_up(incl, d);
                if (lane >= d) incl += y;
            }
            const int pre = incl - pn;                // first virtual index of particle `lane`
            const int tot_m = __shfl(incl, 63);
            const int nchunk = (tot_m + 63) >> 6;
            for (int c = (wv - chunk0) & 3; c < nchunk; c += 4 * KSCAN) {
                int mm[KSCAN];
                int4 bb[KSCAN];
#pragma unroll
                for (int i = 0; i < KSCAN; ++i) {
                    const int v = 64 * (c + 4 * i) + lane;
                    const int vs = min(v, tot_m - 1);
                    // patch holding virtual index vs: the last e < ne with pre[e] <= vs
                    int e = 0;
#pragma unroll
                    for (int st = 32; st; st >>= 1) {
                        const int cand = e + st;
                        const int pc = __shfl(pre, cand & 63);
                        if (cand < ne && pc <= vs) e = cand;
                    }
                    const int m = __shfl(pm0, e) + vs - __shfl(pre, e);
                    mm[i] = v < tot_m ? m : -1;
                    bb[i] = make_int4(0, 0, 0, 0);
                    if (v < tot_m) bb[i] = *(const int4 *)&a.mk[m].b[0];
                }
#pragma unroll
                for (int i = 0; i < KSCAN; ++i) scan(mm[i], bb[i]);
            }
            chunk0 += nchunk;
        }
        drain2(q[lane], lane < qn, q[64 + lane], 64 + lane < qn);
        __syncthreads();
    }

    const uint32_t nxu = (uint32_t)a.nx, sxy = (uint32_t)a.nx * (uint32_t)a.ny;
    using C = typename SF::C;
    using S = typename SF::S;
    constexpr bool SR = sizeof(S) < 8;               // stochastic rounding of the stores
    bool bad = false;
#pragma unroll 1
    for (int kk = 0; kk < TL::N / LBM_THREADS; ++kk) {
        const int ln = tid + LBM_THREADS * kk;
        const int lx = ln % TL::X, lr = ln / TL::X, ly = lr % TL::Y, lz = lr / TL::Y;
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (x >= a.nx || y >= a.ny || z >= a.nz) continue;
        // Populations stay in registers at storage precision; moments and the
        // collision are formed in the compute type C (FP64 for FP32 storage:
        // in a slowly changing region FP32 arithmetic rounds the same way
        // every step and drifts by ~steps x ulp).
        C FB[3] = {0, 0, 0};
        C QB = 0;
        if (has) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const C v = (C)SP::value(acc[c][lr * PXU + lx]);
                if (c < DIM) FB[c] = v;
                else QB = v;
            }
        }
        // 16-bit storage holds the deviation divided by w: the populations stay
        // in that form (WF, WG = w when scaled, else 1), the moments take the
        // weights in their sums, and the collision forms its increments
        // divided by w (the weight factors out of every term of Eqs. lbm2,
        // lbm3, lbm9 and lbm2.5, lbm12.5), so no value is multiplied by w on
        // the way in or divided on the way out.
        constexpr bool SC = SF::SCALED;
        T f[L::Q];
        C g[L::QG];
        pull<DIM, SF, T, C, SC>(a, x, y, z, f, g);
        C fc[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) fc[q] = (C)f[q];
        // raw moments rho - 1, j, S - Tref, summed over opposite pairs
        C drho = (C)(SC ? L::w(0) : 1.0) * fc[0], j[3] = {0, 0, 0};
#pragma unroll
        for (int q = 1; q < L::Q; ++q) {
            const int o = L::opp(q);
            if (q > o) continue;
            const C wq = (C)(SC ? L::w(q) : 1.0);
            const C sp = fc[q] + fc[o], dm = fc[q] - fc[o];
            drho += wq * sp;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                if (L::e(q, d) > 0) j[d] += wq * dm;
                else if (L::e(q, d) < 0) j[d] -= wq * dm;
            }
        }
        C dS = 0;
#pragma unroll
        for (int q = 0; q < L::QG; ++q) dS += (C)(SC ? L::wg(q) : 1.0) * g[q];
        // Sec. 2.1 after Eq. (lbm3.5): T = S + Q_B / 2, u = (j + F / 2) / rho with
        // F = F_B + g beta (T - T_ref) e_up (buoyancy along +y in 2D, +z in 3D).
        const C rho = (C)1 + drho;
        const C dT = dS + (C)0.5 * QB;
        C F[3] = {FB[0], FB[1], FB[2]};
        F[DIM - 1] += (C)a.gbeta * (dT + (C)a.dTb);
        // FP32 compute (16-bit storage): the hardware reciprocal (1 ulp) in
        // place of the correctly rounded division sequence
        C inv;
        if constexpr (std::is_same<C, float>::value) inv = __builtin_amdgcn_rcpf(rho);
        else inv = (C)1 / rho;
        C u[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < DIM; ++d) u[d] = (j[d] + (C)0.5 * F[d]) * inv;
        const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        bad = bad || !(uu <= (C)0.16) || !(rho > (C)0.5 && rho < (C)2);
        const uint32_t n = (uint32_t)z * sxy + (uint32_t)y * nxu + (uint32_t)x;
        if (MACRO) {
            *addr_at(a.macro, n) = (T)rho;
            *addr_at(a.macro + a.Ns, n) = (T)u[0];
            *addr_at(a.macro + 2 * a.Ns, n) = (T)u[1];
            *addr_at(a.macro + 3 * a.Ns, n) = (T)u[2];
            *addr_at(a.macro + 4 * a.Ns, n) = (T)(a.Tref + (double)dT);
            continue;
        }
        const C uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        const C omf = (C)a.omf, gf = (C)a.gf, omg = (C)a.omg, gg = (C)a.gg;
        const uint32_t seed = SR ? node_seed(n, a.seed) : 0u;
        S *fb = (S *)a.fB;
        S *gb = (S *)a.gB;
        // Forced BGK (Eqs. lbm2, lbm3, lbm9) as increments f* - f = src - omega (f - f^eq)
        // over opposite pairs q, q' = -q.  With te = rho e.u, f^eq - w has the
        // even part w (drho - 1.5 rho u.u + 4.5 te e.u) and the odd part 3 w te;
        // the source has the even part w gf (9 e.u e.F - 3 u.F) and the odd
        // part 3 w gf e.F.  So inc(q, q') = P +- M - omega f with
        //   P = w (K3 + e.u (9 gf e.F + 4.5 omega te)),  M = 3 w (gf e.F + omega te),
        //   K3 = omega (drho - 1.5 rho u.u) - 3 gf u.F.
        const C K3 = omf * (drho - (C)1.5 * rho * uu) - (C)3 * gf * uF;
        SF::st_sum(addr_at(fb, n), f[0], (C)(SC ? 1.0 : L::w(0)) * K3 - omf * fc[0], SC ? 1.0 : L::w(0),
                   SR ? sr_bits(seed, 0) : 0u);
#pragma unroll
        for (int q = 1; q < L::Q; ++q) {
            const int o = L::opp(q);
            if (q > o) continue;
            C eu = 0, eF = 0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                if (L::e(q, d) > 0) { eu += u[d]; eF += F[d]; }
                else if (L::e(q, d) < 0) { eu -= u[d]; eF -= F[d]; }
            }
            const C wq = (C)(SC ? 1.0 : L::w(q));
            const C te = rho * eu;
            const C ge = gf * eF;
            const C P = wq * (K3 + eu * ((C)9 * ge + (C)4.5 * omf * te));
            const C M = (C)3 * wq * (ge + omf * te);
            // both arrays of the pair from the pair's first one (q < o)
            S *pb = fb + (size_t)q * a.Ns;
            SF::st_sum(addr_at(pb, n), f[q], (P + M) - omf * fc[q], SC ? 1.0 : L::w(q), SR ? sr_bits(seed, q) : 0u);
            SF::st_sum(addr_at(pb, (uint32_t)(o - q) * (uint32_t)a.Ns + n), f[o], (P - M) - omf * fc[o],
                       SC ? 1.0 : L::w(o), SR ? sr_bits(seed, o) : 0u);
        }
        // Thermal BGK with the linear equilibrium and the heat source
        // (Eqs. lbm2.5, lbm12.5): inc = w (gg Q_B + omega_g dT) +- omega_g w T e.u / c_sg^2 - omega_g g.
        // With temperature on the flow lattice the equilibrium is quadratic
        // (Sec. 2.1): the symmetric part gains omega_g T (4.5 (e.u)^2 - 1.5 u.u).
        const C Tabs = (C)a.Tref + dT;
        const C R = gg * QB + omg * dT + (L::QT ? -(C)1.5 * omg * Tabs * uu : (C)0);
        const C Z = omg * Tabs * (C)L::csg2_inv;
        SF::st_sum(addr_at(gb, n), (T)g[0], (C)(SC ? 1.0 : L::wg(0)) * R - omg * g[0], SC ? 1.0 : L::wg(0),
                   SR ? sr_bits(seed, L::Q) : 0u);
#pragma unroll
        for (int q = 1; q < L::QG; ++q) {
            const int o = L::opp(q);
            if (q > o) continue;
            C eu = 0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                if (L::e(q, d) > 0) eu += u[d];
                else if (L::e(q, d) < 0) eu -= u[d];
            }
            const C wq = (C)(SC ? 1.0 : L::wg(q));
            const C P = wq * (L::QT ? R + (C)4.5 * omg * Tabs * eu * eu : R), M = wq * Z * eu;
            S *pb = gb + (size_t)q * a.Ns;
            SF::st_sum(addr_at(pb, n), (T)g[q], (P + M) - omg * g[q], SC ? 1.0 : L::wg(q),
                       SR ? sr_bits(seed, L::Q + q) : 0u);
            SF::st_sum(addr_at(pb, (uint32_t)(o - q) * (uint32_t)a.Ns + n), (T)g[o], (P - M) - omg * g[o],
                       SC ? 1.0 : L::wg(o), SR ? sr_bits(seed, L::Q + o) : 0u);
        }
    }
    if (bad) atomicOr(a.err, ERR_FIELD);
}

// --------------------------------------------------------------------------
// K2: Lagrangian points of one particle per workgroup.  Generates
// X_l = X_p + r_l and U_l = U_p + Omega x r_l, interpolates the streamed
// moments with the i_max = 2 Lagrange polynomial (Eq. lbm6: multilinear on
// the cell corners, indices clamped at walls / wrapped on periodic axes),
// forms the exchange F_l = 2 (rho_l U_l - j_l) and Q_l = 2 kappa (T_p - T_l)
// (Eqs. lbm7, lbm7.5, lbm8 summed over the bounced directions), writes the
// marker records that K1 spreads, and reduces the reactions of Eq. (lbm13)
// in FP64 in a fixed order.
// --------------------------------------------------------------------------
template <typename T> struct MkArgs {
    LbmArgs<T> lb;
    const DevParticle *part;
    const double4 *tmpl;           // r_l (x, y, z) and A_l
    const int *tmpl_start;
    const double *tmpl_rext;       // largest |r_l| component per template
    const int *mk_start;
    const int *order;              // the particles in cell-list order (a permutation)
    MarkerRec<T> *mk;
    DevReact *react;               // NULL in the macro pass
    double kappa, Tref;
};

__device__ __forceinline__ int clamp_or_wrap(int c, int n, int per)
{
    if (per) { c %= n; if (c < 0) c += n; return c; }
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// Lagrangian-point set-up shared by both gathering modes: position, rigid
// velocity U_l = U_p + Omega x r_l, stencil base and fractions, and the
// cosine-kernel weights stored for K1.
template <int DIM, class T>
__device__ __forceinline__ void marker_setup(const DevParticle &P, const double4 &r4, double *r, double *U,
                                             MarkerRec<T> &rec, double *tt)
{
    r[0] = r4.x; r[1] = r4.y; r[2] = DIM == 3 ? r4.z : 0.0;
    U[0] = P.u[0] + (P.om[1] * r[2] - P.om[2] * r[1]);
    U[1] = P.u[1] + (P.om[2] * r[0] - P.om[0] * r[2]);
    U[2] = DIM == 3 ? P.u[2] + (P.om[0] * r[1] - P.om[1] * r[0]) : 0.0;
    rec.pad = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < DIM) {
            const double X = P.x[d] + r[d];
            const double fl = floor(X);
            rec.b[d] = (int)fl;
            tt[d] = X - fl;
            double wk[4];
            cos_weights(tt[d], wk);
            rec.w[d][0] = (T)wk[0];
            rec.w[d][1] = (T)wk[1];
        } else {
            rec.b[d] = 0; tt[d] = 0;
            rec.w[d][0] = (T)1; rec.w[d][1] = (T)0;      // unused (2D)
        }
    }
}

constexpr int K2_MAXBOX = 16384;    // cells of a particle's stencil box (bitmap)
// distinct stencil nodes whose moments are kept in LDS (larger shells gather
// directly); sized so that several workgroups share a CU
template <class T> struct K2Shell { static constexpr int MAX = sizeof(T) == 8 ? 1024 : 1280; };

// Cubic Lagrange weights of Eq. (lbm6) (i_max = 4) on one axis for a point
// at fraction t of its cell: the nodes b - 1 .. b + 2, l_k(t) = prod_{m != k}
// (t - m) / (k - m) over k, m in {-1, 0, 1, 2}.  (i_max = 2 is 1 - t, t.)
template <int IM>
__device__ __forceinline__ void lagrange_weights(double t, double *w)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = 1.0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (m != k) v *= (t - (m - 1)) / (double)(k - m);
        w[k] = v;
    }
}

template <int DIM, class SF, int IM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_markers(MkArgs<typename SF::T> a)
{
    using T = typename SF::T;
    using C = typename SF::C;
    using L = LatOf<DIM, SF>;
    constexpr int MAXSHELL = K2Shell<T>::MAX;
    __shared__ double wred[4][8];
    __shared__ int spart[256];
    __shared__ uint32_t bits[K2_MAXBOX / 32];
    __shared__ int woff[K2_MAXBOX / 32 + 1];
    __shared__ int cell[MAXSHELL];
    __shared__ T mom[DIM + 2][MAXSHELL];          // rho - 1, j, S - Tref per stencil node
    __shared__ int s_total;
    // Particles in cell-list order, in runs of consecutive ones per XCD (as
    // the lattice tiles): neighbours' stencil rows share 128-byte lines, which
    // are then fetched once into that XCD's L2.  Any permutation gives the
    // same results; an index out of range (a list never built) falls back.
    const int tid = threadIdx.x;
    int p = a.order[xcd_tile(blockIdx.x, gridDim.x)];
    if (p < 0 || p >= gridDim.x) p = blockIdx.x;
    // the particle's loads are issued before the halt check's barrier
    const DevParticle P = a.part[p];
    const int m0 = a.mk_start[p], nm = a.mk_start[p + 1] - m0;
    if (block_halted(a.lb.err)) return;
    if (!centre_ok(P, DIM)) {                      // uniform over the workgroup
        if (tid == 0) atomicOr(a.lb.err, ERR_DOMAIN);
        return;
    }
    const int t0 = a.tmpl_start[P.tmpl];
    const int nn[3] = {a.lb.nx, a.lb.ny, a.lb.nz};

    // Stencil box: the nodes floor(X_l) - LO .. floor(X_l) - LO + IM - 1 of
    // every point (IM Lagrange nodes per axis, Eq. lbm6).
    constexpr int LO = IM == 4 ? 1 : 0;
    constexpr int NCOR = DIM == 3 ? IM * IM * IM : IM * IM;
    const double re = a.tmpl_rext[P.tmpl];
    int bo[3] = {0, 0, 0}, bs[3] = {1, 1, 1};
    for (int d = 0; d < DIM; ++d) {
        bo[d] = (int)floor(P.x[d] - re) - LO;
        bs[d] = (int)floor(P.x[d] + re) - LO + IM - bo[d];
    }
    const int nbox = bs[0] * bs[1] * bs[2];
    const int nwords = (nbox + 31) / 32;
    bool boxed = nbox > 0 && nbox <= K2_MAXBOX;

    // --- 1. mark the stencil nodes, 2. compact them, 3. moments per node ---
    if (boxed) {
        for (int w = tid; w < nwords; w += 256) bits[w] = 0u;
        __syncthreads();
        for (int m = tid; m < nm; m += 256) {
            const double4 r4 = a.tmpl[t0 + m];
            const double r[3] = {r4.x, r4.y, r4.z};
            int u[3] = {0, 0, 0};
            for (int d = 0; d < DIM; ++d) u[d] = (int)floor(P.x[d] + r[d]) - LO - bo[d];
            for (int c = 0; c < NCOR; ++c) {
                const int cx = u[0] + c % IM, cy = u[1] + (c / IM) % IM, cz = u[2] + (DIM == 3 ? c / (IM * IM) : 0);
                const int lin = (cz * bs[1] + cy) * bs[0] + cx;
                atomicOr(&bits[lin >> 5], 1u << (lin & 31));
            }
        }
        __syncthreads();
        // exclusive scan of the per-word counts (Hillis-Steele over 256 partial sums)
        const int per = (nwords + 255) / 256;
        int local = 0;
        for (int w = tid * per; w < min(nwords, (tid + 1) * per); ++w) local += __popc(bits[w]);
        spart[tid] = local;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int v = tid >= off ? spart[tid - off] : 0;
            __syncthreads();
            spart[tid] += v;
            __syncthreads();
        }
        int run = tid == 0 ? 0 : spart[tid - 1];
        for (int w = tid * per; w < min(nwords, (tid + 1) * per); ++w) {
            woff[w] = run;
            run += __popc(bits[w]);
        }
        if (tid == 255) s_total = spart[255];
        __syncthreads();
        boxed = s_total <= MAXSHELL;               // uniform
        if (boxed) {
            for (int w = tid; w < nwords; w += 256) {
                uint32_t b = bits[w];
                int k = woff[w];
                while (b) {
                    const int bit = __ffs(b) - 1;
                    b &= b - 1;
                    cell[k++] = w * 32 + bit;
                }
            }
            __syncthreads();
            const int total = s_total;
            for (int k = tid; k < total; k += 256) {
                const int lin = cell[k];
                int ix[3];
                ix[0] = lin % bs[0];
                ix[1] = (lin / bs[0]) % bs[1];
                ix[2] = lin / (bs[0] * bs[1]);
                for (int d = 0; d < 3; ++d) ix[d] = d < DIM ? clamp_or_wrap(bo[d] + ix[d], nn[d], a.lb.per[d]) : 0;
                T f[L::Q];
                C g[L::QG];
                pull<DIM, SF, T, C>(a.lb, ix[0], ix[1], ix[2], f, g);
                C drho, j[3], dS;
                moments<DIM, L, C>(f, g, drho, j, dS);
                mom[0][k] = (T)drho;
#pragma unroll
                for (int d = 0; d < DIM; ++d) mom[1 + d][k] = (T)j[d];
                mom[DIM + 1][k] = (T)dS;
            }
            __syncthreads();
        }
    }

    // --- 4. interpolation (Eq. lbm6, i_max = 2), exchange, records, reactions ---
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int m = tid; m < nm; m += 256) {
        double r[3], U[3], tt[3];
        MarkerRec<T> rec;
        marker_setup<DIM, T>(P, a.tmpl[t0 + m], r, U, rec, tt);
        const double A = a.tmpl[t0 + m].w;
        // The interpolation and the exchange are formed in FP64 whatever the
        // storage: near a steady state T_p - T_l and rho_l U_l - j_l are small
        // differences of O(1) numbers, and their rounding would act as a
        // systematic source every step.
        double rl = 0, jl[3] = {0, 0, 0}, sl = 0;
        double lw[3][IM];
        if (IM != 2)
#pragma unroll
            for (int d = 0; d < DIM; ++d) lagrange_weights<IM>(tt[d], lw[d]);
#pragma unroll 1
        for (int c = 0; c < NCOR; ++c) {
            double W = 1;
            const int o[3] = {c % IM, (c / IM) % IM, DIM == 3 ? c / (IM * IM) : 0};
#pragma unroll
            for (int d = 0; d < DIM; ++d) W *= IM == 2 ? (o[d] ? tt[d] : 1.0 - tt[d]) : lw[d][o[d]];
            double v[DIM + 2];
            if (boxed) {
                int u[3] = {0, 0, 0};
                for (int d = 0; d < DIM; ++d) u[d] = rec.b[d] + o[d] - LO - bo[d];
                const int lin = (u[2] * bs[1] + u[1]) * bs[0] + u[0];
                const int k = woff[lin >> 5] + __popc(bits[lin >> 5] & ((1u << (lin & 31)) - 1u));
#pragma unroll
                for (int q = 0; q < DIM + 2; ++q) v[q] = (double)mom[q][k];
            } else {
                int ix[3] = {0, 0, 0};
                for (int d = 0; d < DIM; ++d) ix[d] = clamp_or_wrap(rec.b[d] + o[d] - LO, nn[d], a.lb.per[d]);
                T f[L::Q];
                C g[L::QG];
                pull<DIM, SF, T, C>(a.lb, ix[0], ix[1], ix[2], f, g);
                C drho, j[3], dS;
                moments<DIM, L, C>(f, g, drho, j, dS);
                v[0] = (double)drho;
#pragma unroll
                for (int d = 0; d < DIM; ++d) v[1 + d] = (double)j[d];
                v[DIM + 1] = (double)dS;
            }
            rl += W * v[0];
#pragma unroll
            for (int d = 0; d < DIM; ++d) jl[d] += W * v[1 + d];
            sl += W * v[DIM + 1];
        }
        const double rho_l = 1.0 + rl;
        const double dTl = (P.T - a.Tref) - sl;          // T_p - T_l
        double FA[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            FA[d] = d < DIM ? 2.0 * (rho_l * U[d] - jl[d]) * A : 0.0;
            rec.fa[d] = (T)FA[d];
        }
        const double QA = 2.0 * a.kappa * dTl * A;
        rec.qa = (T)QA;
        a.mk[m0 + m] = rec;
        s[0] -= FA[0]; s[1] -= FA[1]; s[2] -= FA[2];
        s[3] -= r[1] * FA[2] - r[2] * FA[1];
        s[4] -= r[2] * FA[0] - r[0] * FA[2];
        s[5] -= r[0] * FA[1] - r[1] * FA[0];
        s[6] += QA;
        s[7] += dTl * A;
    }
    if (!a.react) return;
    // FP64 sums in a fixed order: butterfly within each wave, then the waves
#pragma unroll
    for (int off = 32; off; off >>= 1)
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += __shfl_xor(s[k], off);
    if ((tid & 63) == 0)
#pragma unroll
        for (int k = 0; k < 8; ++k) wred[tid >> 6][k] = s[k];
    __syncthreads();
    if (tid == 0) {
        double t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = (wred[0][k] + wred[1][k]) + (wred[2][k] + wred[3][k]);
        DevReact R;
        R.F[0] = t[0]; R.F[1] = t[1]; R.F[2] = DIM == 3 ? t[2] : 0.0;
        R.tq[0] = DIM == 3 ? t[3] : 0.0; R.tq[1] = DIM == 3 ? t[4] : 0.0; R.tq[2] = t[5];
        R.H = t[6]; R.dTA = t[7];
        a.react[p] = R;
    }
}


// --------------------------------------------------------------------------
// Closure features and targets per particle (the learned closure's inputs and
// outputs; not in the paper).  All dimensionless, so that they carry over
// from a resolved lattice to one coarsened by diffusive scaling:
//   fluid seen by the particle: the raw moments (rho, j, S, no forcing terms)
//     summed over the nodes of the shell 0.75 D <= |x - X_p| <= 1.5 D (a
//     shell in units of D, so the same region on a resolved and on a coarse
//     lattice; inside the body the PIBM fluid moves with the particle and
//     takes its temperature), U_f = sum j / sum rho, T_f = mean S;
//   slip s = U_f - U_p and its frame e1 = s/|s|, e2 = the up axis made
//     normal to e1 (x if s is nearly vertical), e3 = e1 x e2 (2D: e2 = e1
//     turned by +90 degrees);
//   x = [Re_p = |s| D / nu, Gr_p = g beta (T_p - T_f) D^3 / nu^2, phi,
//        T_p - T_f, offsets of the 4 (2D: 6) nearest centres in the frame / D
//        (missing neighbours at 4, 4, 4)], phi = solid volume (area) of the
//        particles whose centres lie within 2 D, over that ball (disk);
//   t = [F.e1, F.e2, F.e3 (2D: 0)] / (3 pi nu D |s|) (drag and lift over the
//       Stokes drag of the slip) and the Nusselt number H / (pi D alpha
//       (T_p - T_f)) in 3D, H / (pi alpha (T_p - T_f)) per unit depth in 2D
//       (0 where |s| or T_p - T_f vanishes), from the point exchange's
//       reactions; the closure inverts these, so its force vanishes with the
//       slip and its heat with the temperature difference.
// One workgroup (256 threads) per particle; shell sums reduced in a fixed
// order; neighbours by a full scan with ties broken by index.
// --------------------------------------------------------------------------
constexpr int FEAT_THREADS = 256;
constexpr int FEAT_NB = 4;                      // neighbours kept (3D); 2D keeps 6

// Cell of a centre along one axis (cells of width cw from -1/2).
__device__ __forceinline__ int cell_coord(double x, int n, int per, int nc, double cw)
{
    double y = x + 0.5;
    if (!(fabs(y) < 1.0e9)) return 0;             // NaN / runaway: not converted (the DEM flags it)
    if (per) { y = fmod(y, (double)n); if (y < 0) y += n; }
    int c = (int)floor(y / cw);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

template <typename T> struct FeatArgs {
    LbmArgs<T> lb;
    const DevParticle *part;
    int np;
    int ncx, ncy, ncz;             // cell list of the current particle state
    double cwx, cwy, cwz;          // cell widths (each >= the largest diameter plus the skin)
    const int *cell_start, *cell_count, *cell_items;
    double nu, alpha, gbeta;
    float *feat;                   // [np][16] raw features (NULL: not stored)
    float *aux;                    // [np][4] slip s and T_f
    uint16_t *xbf;                 // [np][16] normalised BF16 features for the network (NULL: not stored)
    const float *norm;             // mean[16], std[16] of the features
};

template <int DIM>
__device__ __forceinline__ void slip_frame(const double *s, double *e1, double *e2, double *e3)
{
    const double m = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    if (m > 1e-300) { e1[0] = s[0] / m; e1[1] = s[1] / m; e1[2] = s[2] / m; }
    else { e1[0] = 0; e1[1] = 0; e1[2] = 0; e1[DIM - 1] = 1; }
    if (DIM == 2) {
        e2[0] = -e1[1]; e2[1] = e1[0]; e2[2] = 0;
        e3[0] = 0; e3[1] = 0; e3[2] = 1;
        return;
    }
    double up[3] = {0, 0, 1};
    if (fabs(e1[2]) > 0.999) { up[0] = 1; up[2] = 0; }
    const double d = up[0] * e1[0] + up[1] * e1[1] + up[2] * e1[2];
    double v[3] = {up[0] - d * e1[0], up[1] - d * e1[1], up[2] - d * e1[2]};
    const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    e2[0] = v[0] / n; e2[1] = v[1] / n; e2[2] = v[2] / n;
    e3[0] = e1[1] * e2[2] - e1[2] * e2[1];
    e3[1] = e1[2] * e2[0] - e1[0] * e2[2];
    e3[2] = e1[0] * e2[1] - e1[1] * e2[0];
}

template <int DIM, class SF>
__global__ __launch_bounds__(FEAT_THREADS) void k_features(FeatArgs<typename SF::T> a)
{
    using T = typename SF::T;
    using C = double;
    using L = LatOf<DIM, SF>;
    constexpr int NN = DIM == 3 ? 4 : 6;
    // waves 0 .. MW - 1 sum the shell's moments while wave MW finds the
    // neighbours; the two chains of loads overlap and meet at one barrier
    constexpr int MW = FEAT_THREADS / 64 - 1;
    __shared__ double ssum[MW][6];
    __shared__ double s_vol;
    __shared__ int fin_i[6];
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (block_halted(a.lb.err)) return;
    const DevParticle P = a.part[p];
    if (!centre_ok(P, DIM)) {                      // uniform over the workgroup
        if (tid == 0) atomicOr(a.lb.err, ERR_DOMAIN);
        return;
    }
    const int nn[3] = {a.lb.nx, a.lb.ny, a.lb.nz};
    const double D = 2.0 * P.R;
    const double r_in = 0.75 * D, r_out = 1.5 * D, rphi = 2.0 * D;
    // (1) raw moments summed over the shell's nodes, a fixed share per thread
    int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        lo[d] = (int)ceil(P.x[d] - r_out);
        ext[d] = (int)floor(P.x[d] + r_out) - lo[d] + 1;
    }
    bool sane = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) sane = sane && ext[d] >= 1 && ext[d] <= 4096;
    const int nbox = sane ? ext[0] * ext[1] * ext[2] : 0;   // non-finite centre: empty shell
    if (wv < MW) {
        double sm[5] = {0, 0, 0, 0, 0};               // rho, j, S - Tref
        double cnt = 0.0;
        for (int o = tid; o < nbox; o += 64 * MW) {
            int c[3] = {0, 0, 0};
            double r2 = 0.0;
            bool ok = true;
            int oo = o;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const int v0 = lo[d] + oo % ext[d];
                oo /= ext[d];
                const double dx = v0 - P.x[d];
                r2 += dx * dx;
                int v = v0;
                if (a.lb.per[d]) { v %= nn[d]; if (v < 0) v += nn[d]; }
                else if (v < 0 || v >= nn[d]) ok = false;
                c[d] = v;
            }
            if (!ok || r2 < r_in * r_in || r2 > r_out * r_out) continue;
            T f[L::Q];
            C g[L::QG];
            pull<DIM, SF, T, C>(a.lb, c[0], c[1], c[2], f, g);
            C drho, j[3], dS;
            moments<DIM, L, C>(f, g, drho, j, dS);
            sm[0] += 1.0 + drho; sm[1] += j[0]; sm[2] += j[1]; sm[3] += j[2]; sm[4] += dS;
            cnt += 1.0;
        }
#pragma unroll
        for (int off = 32; off; off >>= 1) {
#pragma unroll
            for (int q = 0; q < 5; ++q) sm[q] += __shfl_xor(sm[q], off);
            cnt += __shfl_xor(cnt, off);
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 5; ++q) ssum[wv][q] = sm[q];
            ssum[wv][5] = cnt;
        }
    } else {
        // (2) neighbours.  Every centre within 2 D lies in the 5^d cells around
        // the particle's own (a cell is wider than any diameter), so the solid
        // volume comes from those cells alone.  Their nearest NN (by distance,
        // then index) are the nearest of all particles when the NN-th is closer
        // than two cell widths, the least distance of any centre outside them;
        // otherwise the nearest are searched again over all particles.
        double bd[6];
        int bi[6];
        auto clear = [&]() {
#pragma unroll
            for (int q = 0; q < 6; ++q) { bd[q] = 1e300; bi[q] = 0x7fffffff; }
        };
        auto offer = [&](int jn, double &vol) {
            const DevParticle Q = a.part[jn];
            double d2 = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                double dx = Q.x[d] - P.x[d];
                if (a.lb.per[d]) dx -= nn[d] * rint(dx / nn[d]);
                d2 += dx * dx;
            }
            if (d2 < rphi * rphi)
                vol += DIM == 3 ? (4.0 / 3.0) * M_PI * Q.R * Q.R * Q.R : M_PI * Q.R * Q.R;
            if (jn == p) return;
            if (d2 < bd[NN - 1] || (d2 == bd[NN - 1] && jn < bi[NN - 1])) {
                // sorted insert: replace the last entry and move it up past every
                // larger one (constant indices keep the list in registers)
                bd[NN - 1] = d2; bi[NN - 1] = jn;
#pragma unroll
                for (int q = NN - 1; q > 0; --q)
                    if (bd[q] < bd[q - 1] || (bd[q] == bd[q - 1] && bi[q] < bi[q - 1])) {
                        const double td = bd[q]; bd[q] = bd[q - 1]; bd[q - 1] = td;
                        const int ti = bi[q]; bi[q] = bi[q - 1]; bi[q - 1] = ti;
                    }
            }
        };
        // nearest NN of the lanes' sorted lists: NN rounds of a wave minimum over
        // the list heads; every lane ends with the same nd, ni
        double nd[6];
        int ni[6];
        auto select = [&]() {
#pragma unroll
            for (int r = 0; r < NN; ++r) {
                double md = bd[0];
                int mi = bi[0];
#pragma unroll
                for (int off = 32; off; off >>= 1) {
                    const double od = __shfl_xor(md, off);
                    const int oi = __shfl_xor(mi, off);
                    if (od < md || (od == md && oi < mi)) { md = od; mi = oi; }
                }
                nd[r] = md; ni[r] = mi;
                if (bd[0] == md && bi[0] == mi) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) { bd[q] = bd[q + 1]; bi[q] = bi[q + 1]; }
                    bd[5] = 1e300; bi[5] = 0x7fffffff;
                }
            }
        };
        constexpr int KR = 2;
        const int nc[3] = {a.ncx, a.ncy, DIM == 3 ? a.ncz : 1};
        const double cw[3] = {a.cwx, a.cwy, a.cwz};
        bool centred = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) centred = centred && isfinite(P.x[d]);
        int c0[3] = {0, 0, 0}, span[3] = {1, 1, 1};
        bool full[3] = {true, true, true};
        double bound = 1e300;                          // least distance of a centre outside the cells scanned
        if (centred) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                c0[d] = cell_coord(P.x[d], nn[d], a.lb.per[d], nc[d], cw[d]);
                full[d] = a.lb.per[d] && 2 * KR + 1 >= nc[d];
                span[d] = full[d] ? nc[d] : 2 * KR + 1;
                if (!full[d]) bound = fmin(bound, KR * cw[d] * (1.0 - 1e-9));
            }
        }
        double vol = 0.0;
        clear();
        const int ncs = centred ? span[0] * span[1] * span[2] : 0;
        for (int k = lane; k < ncs; k += 64) {
            int o[3] = {k % span[0], (k / span[0]) % span[1], k / (span[0] * span[1])};
            int cell = 0;
            bool ok = true;
#pragma unroll
            for (int d = 2; d >= 0; --d) {
                int m = o[d];
                if (!full[d]) {
                    m = c0[d] + o[d] - KR;
                    if (a.lb.per[d]) { m %= nc[d]; if (m < 0) m += nc[d]; }
                    else ok = ok && m >= 0 && m < nc[d];
                }
                cell = cell * nc[d] + m;
            }
            if (!ok) continue;
            const int s0 = a.cell_start[cell], e0 = s0 + a.cell_count[cell];
            for (int it = s0; it < e0; ++it) offer(a.cell_items[it], vol);
        }
#pragma unroll
        for (int off = 32; off; off >>= 1) vol += __shfl_xor(vol, off);
        select();
        const bool all_scanned = centred && full[0] && full[1] && full[2];
        const bool exact = all_scanned || (ni[NN - 1] != 0x7fffffff && nd[NN - 1] < bound * bound);
        if (!exact) {
            double dummy = 0.0;
            clear();
            for (int jn = lane; jn < a.np; jn += 64) offer(jn, dummy);
            select();
        }
        if (lane == 0) {
            s_vol = vol;
            for (int q = 0; q < NN; ++q) fin_i[q] = ni[q];
        }
    }
    __syncthreads();
    if (tid != 0) return;
    int ni[6];
    for (int q = 0; q < NN; ++q) ni[q] = fin_i[q];
    const double vtot = s_vol;
    // (3) fluid seen by the particle (waves summed in a fixed order)
    double tot[6] = {0, 0, 0, 0, 0, 0};
    for (int w = 0; w < MW; ++w)
#pragma unroll
        for (int q = 0; q < 6; ++q) tot[q] += ssum[w][q];
    const double irho = tot[0] > 0 ? 1.0 / tot[0] : 0.0;
    const double Uf[3] = {tot[1] * irho, tot[2] * irho, DIM == 3 ? tot[3] * irho : 0.0};
    const double Tf = a.lb.Tref + (tot[5] > 0 ? tot[4] / tot[5] : 0.0);
    double s[3] = {Uf[0] - P.u[0], Uf[1] - P.u[1], DIM == 3 ? Uf[2] - P.u[2] : 0.0};
    double e1[3], e2[3], e3[3];
    slip_frame<DIM>(s, e1, e2, e3);
    const double smag = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    const double dT = P.T - Tf;
    double x[16];
    x[0] = smag * D / a.nu;
    x[1] = a.gbeta * dT * D * D * D / (a.nu * a.nu);
    x[2] = vtot / (DIM == 3 ? (4.0 / 3.0) * M_PI * rphi * rphi * rphi : M_PI * rphi * rphi);
    x[3] = dT;
    for (int q = 0; q < NN; ++q) {
        double o[3] = {4.0, 4.0, 4.0};
        if (ni[q] != 0x7fffffff) {
            double dx[3] = {0, 0, 0};
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                dx[d] = a.part[ni[q]].x[d] - P.x[d];
                if (a.lb.per[d]) dx[d] -= nn[d] * rint(dx[d] / nn[d]);
            }
            o[0] = (dx[0] * e1[0] + dx[1] * e1[1] + dx[2] * e1[2]) / D;
            o[1] = (dx[0] * e2[0] + dx[1] * e2[1] + dx[2] * e2[2]) / D;
            o[2] = (dx[0] * e3[0] + dx[1] * e3[1] + dx[2] * e3[2]) / D;
        }
        if (DIM == 3) { x[4 + 3 * q] = o[0]; x[5 + 3 * q] = o[1]; x[6 + 3 * q] = o[2]; }
        else { x[4 + 2 * q] = o[0]; x[5 + 2 * q] = o[1]; }
    }
    if (a.feat)
        for (int q = 0; q < 16; ++q) a.feat[(size_t)p * 16 + q] = (float)x[q];
    if (a.xbf)
        for (int q = 0; q < 16; ++q) {
            const float v = (float)((x[q] - (double)a.norm[q]) / (double)a.norm[16 + q]);
            const uint32_t u = __float_as_uint(v);
            const uint32_t r = (u & 0x7fffffffu) > 0x7f800000u ? (u | 0x00400000u) : u + 0x7fffu + ((u >> 16) & 1u);
            a.xbf[(size_t)p * 16 + q] = (uint16_t)(r >> 16);
        }
    a.aux[(size_t)p * 4 + 0] = (float)s[0];
    a.aux[(size_t)p * 4 + 1] = (float)s[1];
    a.aux[(size_t)p * 4 + 2] = (float)s[2];
    a.aux[(size_t)p * 4 + 3] = (float)Tf;
}

// Targets of the current state: the reactions of the resolved exchange in
// the slip frame that k_features stored (see above).
template <int DIM>
__global__ void k_targets(const DevParticle *part, int np, const DevReact *react, const float *aux, double nu,
                          double alpha, float *targ)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    double s[3] = {aux[(size_t)p * 4], aux[(size_t)p * 4 + 1], aux[(size_t)p * 4 + 2]};
    double e1[3], e2[3], e3[3];
    slip_frame<DIM>(s, e1, e2, e3);
    const DevReact R = react[p];
    const double D = 2.0 * part[p].R;
    const double smag = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    const double dT = (double)part[p].T - (double)aux[(size_t)p * 4 + 3];
    const double fs = 3.0 * M_PI * nu * D * smag;             // Stokes drag of the slip
    const double hs = M_PI * (DIM == 3 ? D : 1.0) * alpha * dT; // conduction scale of the heat
    const double if_ = fs > 1e-300 ? 1.0 / fs : 0.0, ih = fabs(hs) > 1e-300 ? 1.0 / hs : 0.0;
    targ[(size_t)p * 4 + 0] = (float)((R.F[0] * e1[0] + R.F[1] * e1[1] + R.F[2] * e1[2]) * if_);
    targ[(size_t)p * 4 + 1] = (float)((R.F[0] * e2[0] + R.F[1] * e2[1] + R.F[2] * e2[2]) * if_);
    targ[(size_t)p * 4 + 2] = DIM == 3 ? (float)((R.F[0] * e3[0] + R.F[1] * e3[1] + R.F[2] * e3[2]) * if_) : 0.f;
    targ[(size_t)p * 4 + 3] = (float)(R.H * ih);
}

// The learned closure in the coarse one-point mode: the network's outputs
// (normalised targets) become the hydrodynamic force and heat of each
// particle; its one point carries their reactions to the fluid (F_l A_l =
// -F, Q_l A_l = H) and the DEM receives F and no fluid torque (a point has
// no lever arm).  With `feat` (the raw features) a particle takes the
// network's values only when every feature lies in [range[i], range[16 + i]];
// the others keep the point exchange of Sec. 2.2 (Eqs. lbm7-lbm8, lbm13),
// which the caller ran for every particle before.
template <int DIM, class T>
__global__ void k_closure(const DevParticle *part, int np, const float *y, const float *norm, const float *aux,
                          const float *feat, const float *range, double nu, double alpha, double kappa,
                          MarkerRec<T> *mk, DevReact *react, int *err)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np || halted(err)) return;
    const DevParticle P = part[p];
    if (!centre_ok(P, DIM)) {
        atomicOr(err, ERR_DOMAIN);
        return;
    }
    if (feat) {
        // a feature outside the range (or not a number): the particle keeps
        // the point exchange's record and reactions, written before
        bool in = true;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float v = feat[(size_t)p * 16 + i];
            in = in && v >= range[i] && v <= range[16 + i];
        }
        if (!in) return;
    }
    double yv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) yv[q] = (double)y[(size_t)p * 4 + q] * (double)norm[36 + q] + (double)norm[32 + q];
    double s[3] = {aux[(size_t)p * 4], aux[(size_t)p * 4 + 1], aux[(size_t)p * 4 + 2]};
    double e1[3], e2[3], e3[3];
    slip_frame<DIM>(s, e1, e2, e3);
    const double D = 2.0 * P.R;
    const double fs = 3.0 * M_PI * nu * D * sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    const double dT = P.T - (double)aux[(size_t)p * 4 + 3];
    double F[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) F[c] = (yv[0] * e1[c] + yv[1] * e2[c] + (DIM == 3 ? yv[2] * e3[c] : 0.0)) * fs;
    if (DIM == 2) F[2] = 0.0;
    const double H = yv[3] * M_PI * (DIM == 3 ? D : 1.0) * alpha * dT;
    MarkerRec<T> rec;
    double r[3], U[3], tt[3];
    marker_setup<DIM, T>(P, make_double4(0.0, 0.0, 0.0, 0.0), r, U, rec, tt);
#pragma unroll
    for (int c = 0; c < 3; ++c) rec.fa[c] = (T)(-F[c]);
    rec.qa = (T)H;
    mk[p] = rec;
    DevReact R;
#pragma unroll
    for (int c = 0; c < 3; ++c) { R.F[c] = F[c]; R.tq[c] = 0.0; }
    R.H = H;
    // the exchange's sum (T_p - T_l) A that would give this heat: H = 2 kappa_T sum (T_p - T_l) A
    R.dTA = kappa != 0.0 ? H / (2.0 * kappa) : 0.0;
    react[p] = R;
}

// --------------------------------------------------------------------------
// K3: bin particles into lattice tiles (integer counting sort).  A particle
// lands in every tile its markers' spreading footprints can touch: nodes
// floor(X - rext) - 1 .. floor(X + rext) + 2 per axis.
// --------------------------------------------------------------------------
struct BinArgs {
    int dim, nx, ny, nz, per[3];
    int TX, TY, TZ, ntx, nty, ntz;
    int np;
    const DevParticle *part;
    const int *tp_start;           // ntmpl + 1: first patch of each template
    const double *tp_box;          // 6 per patch: least and greatest offset per axis
    const int *gp_base;            // np + 1: first patch id of each particle
    const int *gp_start;           // first point record of each patch (one more entry: the total)
    long long cap;                 // capacity of tile_items
    int *tile_count, *tile_start, *tile_fill;
    int2 *tile_items;              // (first point record, point count) of each listed patch
    int *err;
};

constexpr int MAXT_AXIS = 32;     // particles whose footprint spans more tiles per axis are refused

// Tiles along one axis that hold a node of lo .. hi (wrapped on a periodic
// axis, clipped otherwise): first .. first + cntA - 1, then 0 .. cnt - cntA
// - 1 (the part of a wrapped range that lies below `first`), each once.
struct AxisRun { int first, cntA, cnt; };
__device__ inline AxisRun axis_run(int lo, int hi, int n, int per, int T)
{
    AxisRun r{0, 0, 0};
    if (!per) {
        const int a = max(lo, 0), b = min(hi, n - 1);
        if (a <= b) { r.first = a / T; r.cntA = r.cnt = b / T - a / T + 1; }
        return r;
    }
    int m = lo % n;
    if (m < 0) m += n;
    r.first = m / T;
    if (hi - lo + 1 >= n) {                        // every node
        r.cntA = (n - 1) / T - r.first + 1;
        r.cnt = r.cntA + r.first;
        return r;
    }
    const int e = m + (hi - lo);
    if (e < n) { r.cntA = r.cnt = e / T - r.first + 1; return r; }
    r.cntA = (n - 1) / T - r.first + 1;
    r.cnt = r.cntA + min((e - n) / T, r.first - 1) + 1;
    return r;
}
__device__ __forceinline__ int axis_tile(const AxisRun &r, int i) { return i < r.cntA ? r.first + i : i - r.cntA; }

// One wave per particle.  Its points are grouped in patches (boxes of
// offsets from the centre); the tiles of a patch are those its points'
// footprints (nodes floor(X) - 1 .. floor(X) + 2 per axis) can reach.  The
// lanes take the particle's (patch, tile) pairs in turn; an item names the
// particle's patch, so the lattice kernel scans only the points near a tile.
constexpr int BIN_THREADS = 256;
template <bool FILL>
__device__ __forceinline__ void bin_particle(const BinArgs &a, int p, int lane)
{
    if (halted(a.err)) return;                     // uniform over the wave, as every early return here
    const DevParticle P = a.part[p];
    // a non-finite or runaway centre would give meaningless loop bounds
    if (!centre_ok(P, a.dim)) {
        if (!FILL && lane == 0) atomicOr(a.err, ERR_DOMAIN);
        return;
    }
    const int k0 = a.tp_start[P.tmpl], nk = a.tp_start[P.tmpl + 1] - k0;
    const int g0 = a.gp_base[p];
    const int nn[3] = {a.nx, a.ny, a.nz}, TT[3] = {a.TX, a.TY, a.TZ};
    for (int kb = 0; kb < nk; kb += 64) {
        // lane = patch kb + lane: its node range and tile count per axis
        const int k = kb + lane;
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, ncomb = 0;
        if (k < nk) {
            const double *bx = a.tp_box + 6 * (size_t)(k0 + k);
            ncomb = 1;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (d < a.dim) {
                    lo[d] = (int)floor(P.x[d] + bx[d]) - 1;
                    hi[d] = (int)floor(P.x[d] + bx[3 + d]) + 2;
                    ncomb *= axis_run(lo[d], hi[d], nn[d], a.per[d], TT[d]).cnt;
                }
        }
        int incl = ncomb;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        const int pre = incl - ncomb, tot = __shfl(incl, 63);
        for (int f0 = 0; f0 < tot; f0 += 64) {
            const int f = f0 + lane;
            // the patch holding pair f: the last lane e with pre[e] <= f
            int e = 0;
#pragma unroll
            for (int st = 32; st; st >>= 1) {
                const int cand = e + st;
                if (__shfl(pre, cand) <= f) e = cand;
            }
            int elo[3], ehi[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) { elo[d] = __shfl(lo[d], e); ehi[d] = __shfl(hi[d], e); }
            const int c = f - __shfl(pre, e);
            if (f >= tot) continue;
            AxisRun r[3] = {{0, 1, 1}, {0, 1, 1}, {0, 1, 1}};
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (d < a.dim) r[d] = axis_run(elo[d], ehi[d], nn[d], a.per[d], TT[d]);
            const int ix = c % r[0].cnt, iy = (c / r[0].cnt) % r[1].cnt, iz = c / (r[0].cnt * r[1].cnt);
            const int t = (axis_tile(r[2], iz) * a.nty + axis_tile(r[1], iy)) * a.ntx + axis_tile(r[0], ix);
            if (FILL) {
                const int pos = atomicAdd(&a.tile_fill[t], 1);
                const long long at = (long long)a.tile_start[t] + pos;
                if (at < a.cap) {
                    // the patch's range of point records, so that the lattice kernel
                    // reads it with the list instead of one dependent load later
                    const int g = g0 + kb + e;
                    a.tile_items[at] = make_int2(a.gp_start[g], a.gp_start[g + 1] - a.gp_start[g]);
                }
                else atomicOr(a.err, ERR_TILES);
            } else {
                atomicAdd(&a.tile_count[t], 1);
            }
        }
    }
}

template <bool FILL>
__global__ __launch_bounds__(BIN_THREADS) void k_bin(BinArgs a)
{
    const int p = blockIdx.x * (BIN_THREADS / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (p < a.np) bin_particle<FILL>(a, p, lane);
}

// One thread per patch: global patch g (patch g - base[p] of particle p's
// template, base = the particles' first patch ids, np + 1 entries) counted
// into or listed in the tiles its points' footprints can reach, as in
// bin_particle.  The ranges are read with atomic loads: they were written by
// other waves of the same workgroup in this launch.
constexpr int BIN_ONE_WG_PARTICLES = 256, BIN_ONE_WG_TILES = 16384;
template <bool FILL>
__device__ __forceinline__ void bin_patch(const BinArgs &a, int g, const int *base)
{
    int p = 0;                                     // the last particle with base[p] <= g
#pragma unroll
    for (int st = BIN_ONE_WG_PARTICLES / 2; st; st >>= 1)
        if (p + st < a.np && base[p + st] <= g) p += st;
    const DevParticle P = a.part[p];
    const int k = g - base[p];
    if (!centre_ok(P, a.dim)) {
        if (!FILL && k == 0) atomicOr(a.err, ERR_DOMAIN);
        return;
    }
    const double *bx = a.tp_box + 6 * (size_t)(a.tp_start[P.tmpl] + k);
    const int nn[3] = {a.nx, a.ny, a.nz}, TT[3] = {a.TX, a.TY, a.TZ};
    AxisRun r[3] = {{0, 1, 1}, {0, 1, 1}, {0, 1, 1}};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (d < a.dim)
            r[d] = axis_run((int)floor(P.x[d] + bx[d]) - 1, (int)floor(P.x[d] + bx[3 + d]) + 2, nn[d], a.per[d], TT[d]);
    const int ncomb = r[0].cnt * r[1].cnt * r[2].cnt;
    int2 item = make_int2(0, 0);
    if (FILL) item = make_int2(a.gp_start[g], a.gp_start[g + 1] - a.gp_start[g]);
    for (int c = 0; c < ncomb; ++c) {
        const int ix = c % r[0].cnt, iy = (c / r[0].cnt) % r[1].cnt, iz = c / (r[0].cnt * r[1].cnt);
        const int t = (axis_tile(r[2], iz) * a.nty + axis_tile(r[1], iy)) * a.ntx + axis_tile(r[0], ix);
        if (FILL) {
            const int pos = atomicAdd(&a.tile_fill[t], 1);
            const long long at = (long long)__atomic_load_n(&a.tile_start[t], __ATOMIC_RELAXED) + pos;
            if (at < a.cap) a.tile_items[at] = item;
            else atomicOr(a.err, ERR_TILES);
        } else {
            atomicAdd(&a.tile_count[t], 1);
        }
    }
}

__device__ __forceinline__ void alloc_one_wg(const int *count, int *start, int *fill, int n, int *total);

// Few particles and tiles: the four phases of binning (zero, count, ranges,
// fill: k_zero2, k_bin, k_alloc, k_bin) in one workgroup of ONE_WG threads,
// one thread per patch, barriers between the phases.  Before each barrier a
// wave waits until its global stores and atomics are done, so that the next
// phase's atomics and loads in other waves find them.  The lists hold the
// same items as k_bin's, in another order within a tile, which no result
// depends on.
__global__ __launch_bounds__(1024) void k_bin_one_wg(BinArgs a, int nt, int *total)
{
    __shared__ int base[BIN_ONE_WG_PARTICLES + 1];
    const int tid = threadIdx.x;
    if (block_halted(a.err)) return;
    for (int i = tid; i < nt; i += 1024) a.tile_count[i] = 0;
    if (tid == 0) *total = 0;
    for (int p = tid; p <= a.np; p += 1024) base[p] = a.gp_base[p];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int npatch = base[a.np];
    for (int g = tid; g < npatch; g += 1024) bin_patch<false>(a, g, base);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    alloc_one_wg(a.tile_count, a.tile_start, a.tile_fill, nt, total);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int g = tid; g < npatch; g += 1024) bin_patch<true>(a, g, base);
}

__global__ void k_fill_int(int *p, long long n, int v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Disjoint ranges of the items array for the bins: start[i] such that the
// ranges [start[i], start[i] + count[i]) tile [0, sum count) in some order
// (a wave prefix sum and one atomic per wave).  Every user of the lists is
// independent of their order.  Also clears fill[i] for the scatter pass.
__global__ __launch_bounds__(256) void k_alloc(const int *count, int *start, int *fill, int n, int *total)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, lane = threadIdx.x & 63;
    const int c = i < n ? count[i] : 0;
    int incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    int base = 0;
    if (lane == 63) base = atomicAdd(total, incl);
    base = __shfl(base, 63);
    if (i < n) {
        start[i] = base + incl - c;
        fill[i] = 0;
    }
}

// Zero two integer arrays in one launch.
__global__ void k_zero2(int *a, long long na, int *b, long long nb)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < na + nb; i += (long long)gridDim.x * blockDim.x) {
        if (i < na) a[i] = 0;
        else b[i - na] = 0;
    }
}


// --------------------------------------------------------------------------
// K4: DEM cell list and per-particle Verlet list (candidates within
// R_i + R_j + skin, ascending index for a fixed force-summation order).
// --------------------------------------------------------------------------
constexpr int MAXN = 32;           // neighbour candidates per particle
constexpr int MAXC = 16;           // contact slots per particle (particles + walls)

struct DemArgs {
    int dim, nx, ny, nz, per[3];
    int np;
    int ncx, ncy, ncz;
    double cwx, cwy, cwz;          // cell widths
    double skin;
    const DevParticle *cur;
    DevParticle *nxt;
    const DevReact *react;
    int *cell_count, *cell_start, *cell_fill, *cell_items;
    int *nbr, *nbr_n;
    double *xref;                  // 3 per particle: positions at list build
    const int *hid_in; const double *hxi_in; const int *hn_in;
    int *hid_out; double *hxi_out; int *hn_out;
    double E, G, mu, dts;
    double gravity, beta_p, c_r, Tref;
    int last;                      // last sub-step: apply the thermosensitive update
    int *err;
};

template <bool FILL>
__device__ __forceinline__ void cell_particle(const DemArgs &a, int p)
{
    if (halted(a.err)) return;
    const DevParticle P = a.cur[p];
    const int cx = cell_coord(P.x[0], a.nx, a.per[0], a.ncx, a.cwx);
    const int cy = cell_coord(P.x[1], a.ny, a.per[1], a.ncy, a.cwy);
    const int cz = a.dim == 3 ? cell_coord(P.x[2], a.nz, a.per[2], a.ncz, a.cwz) : 0;
    const int c = (cz * a.ncy + cy) * a.ncx + cx;
    if (FILL) {
        const int pos = atomicAdd(&a.cell_fill[c], 1);
        a.cell_items[a.cell_start[c] + pos] = p;
    } else {
        atomicAdd(&a.cell_count[c], 1);
    }
}

template <bool FILL>
__global__ void k_cells(DemArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < a.np) cell_particle<FILL>(a, p);
}

// Few particles: the four phases of the cell list (zero, count, ranges,
// fill: k_zero2, k_cells, k_alloc, k_cells) in one workgroup, barriers
// between the phases.  The list is the same up to the order of items within
// a cell, which no result depends on.  Counts built by device-scope atomics
// are read back with atomic loads.
constexpr int ONE_WG = 1024;
__device__ __forceinline__ void alloc_one_wg(const int *count, int *start, int *fill, int n, int *total)
{
    const int tid = threadIdx.x, lane = tid & 63;
    for (int b = 0; b < n; b += ONE_WG) {
        const int i = b + tid;
        const int c = i < n ? __atomic_load_n(&count[i], __ATOMIC_RELAXED) : 0;
        int incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        int base = 0;
        if (lane == 63) base = atomicAdd(total, incl);
        base = __shfl(base, 63);
        if (i < n) {
            start[i] = base + incl - c;
            fill[i] = 0;
        }
    }
}

// The cell list and the tile lists of one particle state in one workgroup
// (few particles, cells and tiles): the phases of k_cells_one_wg and
// k_bin_one_wg interleaved, four barriers for both.
__global__ __launch_bounds__(ONE_WG) void k_cells_bin_one_wg(DemArgs d, int ncells, int *ctotal, BinArgs b, int nt,
                                                             int *btotal)
{
    __shared__ int base[BIN_ONE_WG_PARTICLES + 1];
    const int tid = threadIdx.x;
    if (block_halted(b.err)) return;
    for (int i = tid; i < ncells; i += ONE_WG) d.cell_count[i] = 0;
    for (int i = tid; i < nt; i += ONE_WG) b.tile_count[i] = 0;
    if (tid == 0) { *ctotal = 0; *btotal = 0; }
    for (int p = tid; p <= b.np; p += ONE_WG) base[p] = b.gp_base[p];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int npatch = base[b.np];
    for (int p = tid; p < d.np; p += ONE_WG) cell_particle<false>(d, p);
    for (int g = tid; g < npatch; g += ONE_WG) bin_patch<false>(b, g, base);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    alloc_one_wg(d.cell_count, d.cell_start, d.cell_fill, ncells, ctotal);
    alloc_one_wg(b.tile_count, b.tile_start, b.tile_fill, nt, btotal);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int p = tid; p < d.np; p += ONE_WG) cell_particle<true>(d, p);
    for (int g = tid; g < npatch; g += ONE_WG) bin_patch<true>(b, g, base);
}

__global__ __launch_bounds__(ONE_WG) void k_cells_one_wg(DemArgs a, int ncells, int *total)
{
    const int tid = threadIdx.x;
    for (int i = tid; i < ncells; i += ONE_WG) a.cell_count[i] = 0;
    if (tid == 0) *total = 0;
    __syncthreads();
    for (int p = tid; p < a.np; p += ONE_WG) cell_particle<false>(a, p);
    __syncthreads();
    alloc_one_wg(a.cell_count, a.cell_start, a.cell_fill, ncells, total);
    __syncthreads();
    for (int p = tid; p < a.np; p += ONE_WG) cell_particle<true>(a, p);
}

__device__ __forceinline__ void min_image(const DemArgs &a, const double *xi, const double *xj, double *d)
{
    const int nn[3] = {a.nx, a.ny, a.nz};
    for (int c = 0; c < 3; ++c) {
        d[c] = xj[c] - xi[c];
        if (c == 2 && a.dim == 2) { d[c] = 0; continue; }
        if (a.per[c]) {
            const double L = nn[c];
            if (d[c] > 0.5 * L) d[c] -= L;
            else if (d[c] < -0.5 * L) d[c] += L;
        }
    }
}

__device__ inline int axis_cells(int c, int nc, int per, int *out)
{
    int cnt = 0;
    for (int o = -1; o <= 1; ++o) {
        int m = c + o;
        if (per) { m %= nc; if (m < 0) m += nc; }
        else if (m < 0 || m >= nc) continue;
        bool dup = false;
        for (int k = 0; k < cnt; ++k) dup = dup || out[k] == m;
        if (!dup) out[cnt++] = m;
    }
    return cnt;
}

// One wave per particle: lane c scans cell c of the 3^d neighbourhood; the
// hits are gathered and kept in ascending order.
constexpr int NBR_THREADS = 256;
__global__ __launch_bounds__(NBR_THREADS) void k_neighbours(DemArgs a)
{
    __shared__ int hits[NBR_THREADS / 64][MAXN + 64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * (NBR_THREADS / 64) + wv;
    if (i >= a.np || halted(a.err)) return;
    const DevParticle P = a.cur[i];
    const int cx = cell_coord(P.x[0], a.nx, a.per[0], a.ncx, a.cwx);
    const int cy = cell_coord(P.x[1], a.ny, a.per[1], a.ncy, a.cwy);
    const int cz = a.dim == 3 ? cell_coord(P.x[2], a.nz, a.per[2], a.ncz, a.cwz) : 0;
    int lx[3], ly[3], lz[3];
    const int nx = axis_cells(cx, a.ncx, a.per[0], lx);
    const int ny = axis_cells(cy, a.ncy, a.per[1], ly);
    int nz = 1;
    lz[0] = 0;
    if (a.dim == 3) nz = axis_cells(cz, a.ncz, a.per[2], lz);
    int *h = hits[wv];
    int n = 0;                                    // wave-uniform
    bool over = false;
    const int ncell = nx * ny * nz;
    const int cell = lane < ncell ? (lz[lane / (nx * ny)] * a.ncy + ly[(lane / nx) % ny]) * a.ncx + lx[lane % nx] : 0;
    int s = lane < ncell ? a.cell_start[cell] : 0;
    const int e = lane < ncell ? s + a.cell_count[cell] : 0;
    // one candidate per lane at a time; the lanes advance through their cells together
    while (__ballot(s < e)) {
        bool hit = false;
        int j = -1;
        if (s < e) {
            j = a.cell_items[s++];
            if (j != i) {
                const DevParticle Q = a.cur[j];
                double d[3];
                min_image(a, P.x, Q.x, d);
                const double lim = P.R + Q.R + a.skin;
                hit = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < lim * lim;
            }
        }
        const unsigned long long m = __ballot(hit);
        const int k = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (hit && n + k < MAXN) h[n + k] = j;
        const int cnt = __popcll(m);
        if (n + cnt > MAXN) over = true;
        n = min(n + cnt, MAXN);
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        for (int q = 1; q < n; ++q) {             // ascending order (insertion)
            const int v = h[q];
            int r = q - 1;
            while (r >= 0 && h[r] > v) { h[r + 1] = h[r]; --r; }
            h[r + 1] = v;
        }
    }
    __builtin_amdgcn_wave_barrier();
    for (int q = lane; q < n; q += 64) a.nbr[(size_t)i * MAXN + q] = h[q];
    if (lane == 0) {
        a.nbr_n[i] = n;
        a.xref[3 * i] = P.x[0]; a.xref[3 * i + 1] = P.x[1]; a.xref[3 * i + 2] = P.x[2];
        if (over) atomicOr(a.err, ERR_NEIGHBOURS);
    }
}

// --------------------------------------------------------------------------
// K5: one DEM sub-step per launch, state double-buffered (cur -> nxt).
// Hertz normal force F_n = 4/3 E* sqrt(R*) delta^(3/2) (Sec. 2.3);
// tangential spring with stiffness 8 G* sqrt(R* delta) (the
// Mindlin-Deresiewicz increment in its no-slip limit) capped by mu F_n, with
// G* = (1 - nu) E* / (2 (2 - nu)) for equal materials; semi-implicit Euler
// of Eq. (demgov) with the particle mass on the gravity term.
// --------------------------------------------------------------------------
__device__ inline void contact(const DemArgs &a, double Ri, const double *n, double delta, double Rstar,
                               const double *vrel, const double *xi_old, double *F, double *Tq, double *xi)
{
    const double Fn = 4.0 / 3.0 * a.E * sqrt(Rstar) * delta * sqrt(delta);
    const double vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    const double vt[3] = {vrel[0] - vn * n[0], vrel[1] - vn * n[1], vrel[2] - vn * n[2]};
    double x[3] = {xi_old[0], xi_old[1], xi_old[2]};
    const double xn = x[0] * n[0] + x[1] * n[1] + x[2] * n[2];
    for (int c = 0; c < 3; ++c) x[c] = x[c] - xn * n[c] + vt[c] * a.dts;
    const double kt = 8.0 * a.G * sqrt(Rstar * delta);
    double Ft[3] = {-kt * x[0], -kt * x[1], -kt * x[2]};
    const double ft = sqrt(Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2]);
    const double cap = a.mu * Fn;
    if (ft > cap) {
        const double sc = cap / ft;
        for (int c = 0; c < 3; ++c) { Ft[c] *= sc; x[c] = -Ft[c] / kt; }
    }
    for (int c = 0; c < 3; ++c) { F[c] = -Fn * n[c] + Ft[c]; xi[c] = x[c]; }
    const double rn[3] = {Ri * n[0], Ri * n[1], Ri * n[2]};
    Tq[0] = rn[1] * Ft[2] - rn[2] * Ft[1];
    Tq[1] = rn[2] * Ft[0] - rn[0] * Ft[2];
    Tq[2] = rn[0] * Ft[1] - rn[1] * Ft[0];
}

__device__ __forceinline__ void dem_particle(const DemArgs &a, int i)
{
    const DevParticle P = a.cur[i];
    if (halted(a.err)) {
        a.nxt[i] = P;                  // keep both particle copies identical
        a.hn_out[i] = a.hn_in[i];
        for (int s = 0; s < a.hn_in[i] && s < MAXC; ++s) {
            const size_t k = (size_t)i * MAXC + s;
            a.hid_out[k] = a.hid_in[k];
            a.hxi_out[3 * k] = a.hxi_in[3 * k]; a.hxi_out[3 * k + 1] = a.hxi_in[3 * k + 1]; a.hxi_out[3 * k + 2] = a.hxi_in[3 * k + 2];
        }
        return;
    }
    const int dim = a.dim;
    const int nold = a.hn_in[i];
    double Fc[3] = {0, 0, 0}, Tc[3] = {0, 0, 0};
    int nnew = 0;
    bool over = false;
    const size_t hb = (size_t)i * MAXC;
    auto find_old = [&](int partner, double *xo) {
        xo[0] = xo[1] = xo[2] = 0.0;
        for (int s = 0; s < nold; ++s)
            if (a.hid_in[hb + s] == partner) {
                xo[0] = a.hxi_in[3 * (hb + s)]; xo[1] = a.hxi_in[3 * (hb + s) + 1]; xo[2] = a.hxi_in[3 * (hb + s) + 2];
                return;
            }
    };
    auto record = [&](int partner, const double *xi) {
        if (nnew < MAXC) {
            a.hid_out[hb + nnew] = partner;
            a.hxi_out[3 * (hb + nnew)] = xi[0]; a.hxi_out[3 * (hb + nnew) + 1] = xi[1]; a.hxi_out[3 * (hb + nnew) + 2] = xi[2];
            ++nnew;
        } else over = true;
    };
    const double wiP[3] = {P.om[0], P.om[1], P.om[2]};
    const int nn = a.nbr_n[i];
    for (int k = 0; k < nn; ++k) {
        const int j = a.nbr[(size_t)i * MAXN + k];
        const DevParticle Q = a.cur[j];
        double d[3];
        min_image(a, P.x, Q.x, d);
        const double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (!(dist < P.R + Q.R)) continue;
        const double n[3] = {d[0] / dist, d[1] / dist, d[2] / dist};
        const double delta = P.R + Q.R - dist;
        const double Rstar = P.R * Q.R / (P.R + Q.R);
        const double ri[3] = {P.R * n[0], P.R * n[1], P.R * n[2]};
        const double rj[3] = {Q.R * n[0], Q.R * n[1], Q.R * n[2]};
        const double wi[3] = {wiP[1] * ri[2] - wiP[2] * ri[1], wiP[2] * ri[0] - wiP[0] * ri[2], wiP[0] * ri[1] - wiP[1] * ri[0]};
        const double wj[3] = {Q.om[1] * rj[2] - Q.om[2] * rj[1], Q.om[2] * rj[0] - Q.om[0] * rj[2], Q.om[0] * rj[1] - Q.om[1] * rj[0]};
        double vrel[3];
        for (int c = 0; c < 3; ++c) vrel[c] = (P.u[c] - Q.u[c]) + (wi[c] + wj[c]);
        double xo[3], F[3], T[3], xn[3];
        find_old(j, xo);
        contact(a, P.R, n, delta, Rstar, vrel, xo, F, T, xn);
        for (int c = 0; c < 3; ++c) { Fc[c] += F[c]; Tc[c] += T[c]; }
        record(j, xn);
    }
    // walls; loops over axes run to 3 with a guard so that every index is a
    // constant and the particle records stay in registers
    const int nn3[3] = {a.nx, a.ny, a.nz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (ax >= dim || a.per[ax]) continue;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const double gap = side == 0 ? P.x[ax] + 0.5 : (nn3[ax] - 0.5) - P.x[ax];
            const double delta = P.R - gap;
            if (!(delta > 0)) continue;
            double n[3] = {0, 0, 0};
            n[ax] = side == 0 ? -1.0 : 1.0;
            const double ri[3] = {P.R * n[0], P.R * n[1], P.R * n[2]};
            const double wi[3] = {wiP[1] * ri[2] - wiP[2] * ri[1], wiP[2] * ri[0] - wiP[0] * ri[2], wiP[0] * ri[1] - wiP[1] * ri[0]};
            double vrel[3];
            for (int c = 0; c < 3; ++c) vrel[c] = P.u[c] + wi[c];
            const int partner = -1 - (2 * ax + side);
            double xo[3], F[3], T[3], xn[3];
            find_old(partner, xo);
            contact(a, P.R, n, delta, P.R, vrel, xo, F, T, xn);
            for (int c = 0; c < 3; ++c) { Fc[c] += F[c]; Tc[c] += T[c]; }
            record(partner, xn);
        }
    }
    a.hn_out[i] = nnew;
    DevParticle O = P;
    const DevReact Rh = a.react[i];
    if (!(P.flags & 1)) {
        const double pi = 3.14159265358979323846;
        const double V = dim == 2 ? pi * P.R * P.R : 4.0 / 3.0 * pi * P.R * P.R * P.R;
        const double m = P.rho_r * V;
        const double I = dim == 2 ? 0.5 * m * P.R * P.R : 0.4 * m * P.R * P.R;
        double rho_p = P.rho_r;
        if (P.flags & 2) rho_p = P.rho_r * (1.0 - a.beta_p * (P.T - a.Tref));
        const double gup = -a.gravity * (1.0 - 1.0 / rho_p);     // along the last axis
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (c >= dim) continue;
            const double gv = c == dim - 1 ? gup : 0.0;
            O.u[c] = P.u[c] + a.dts * ((Rh.F[c] + Fc[c]) / m + gv);
            O.x[c] = P.x[c] + a.dts * O.u[c];
        }
        if (dim == 2) {
            O.om[2] = P.om[2] + a.dts * (Rh.tq[2] + Tc[2]) / I;
            O.th[2] = P.th[2] + a.dts * O.om[2];
        } else {
            for (int c = 0; c < 3; ++c) {
                O.om[c] = P.om[c] + a.dts * (Rh.tq[c] + Tc[c]) / I;
                O.th[c] = P.th[c] + a.dts * O.om[c];
            }
        }
    }
    if (a.last && (P.flags & 2)) {
        const double pi = 3.14159265358979323846;
        const double V = dim == 2 ? pi * P.R * P.R : 4.0 / 3.0 * pi * P.R * P.R * P.R;
        O.T = P.T - Rh.H / (P.rho_r * a.c_r * V);
    }
    a.nxt[i] = O;
    // watchdog: stale neighbour list, NaN, centre beyond a wall
    double dd[3];
    const double xr[3] = {a.xref[3 * i], a.xref[3 * i + 1], a.xref[3 * i + 2]};
    min_image(a, xr, O.x, dd);
    int e = 0;
    if (!(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2] <= 0.25 * a.skin * a.skin)) e |= ERR_STALE;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (c >= dim) continue;
        if (!a.per[c] && !(O.x[c] > -0.5 && O.x[c] < nn3[c] - 0.5)) e |= ERR_DOMAIN;
        if (!(fabs(O.x[c]) < 1.0e8) || !(fabs(O.u[c]) < 1.0e8)) e |= ERR_DOMAIN;
    }
    if (over) e |= ERR_CONTACTS;
    if (e) atomicOr(a.err, e);
}

// One sub-step per launch, one thread per particle.
__global__ void k_dem(DemArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.np) dem_particle(a, i);
}

// Every sub-step in one workgroup, one thread per particle (np <=
// DEM_ONE_WG): the particle and contact-history buffers alternate as between
// k_dem launches and a barrier separates the sub-steps.  Each particle reads
// only the previous sub-step's buffers and writes its own slots, so the
// results are those of k_dem; for a few hundred particles one launch costs
// less than one per sub-step.
struct DemOneWg {
    DemArgs a;                     // cur / nxt and the history pointers are set per sub-step
    DevParticle *part[2];          // part[0] holds the state at the first sub-step
    int *hid[2], *hn[2];           // hid[0], hn[0], hxi[0]: the history at the first sub-step
    double *hxi[2];
    int n_sub;
};
constexpr int DEM_ONE_WG = 512;

__global__ __launch_bounds__(DEM_ONE_WG) void k_dem_one_wg(DemOneWg f)
{
    for (int s = 0; s < f.n_sub; ++s) {
        DemArgs a = f.a;
        const int c = s & 1;
        a.cur = f.part[c];
        a.nxt = f.part[c ^ 1];
        a.hid_in = f.hid[c]; a.hxi_in = f.hxi[c]; a.hn_in = f.hn[c];
        a.hid_out = f.hid[c ^ 1]; a.hxi_out = f.hxi[c ^ 1]; a.hn_out = f.hn[c ^ 1];
        a.last = s == f.n_sub - 1;
        if ((int)threadIdx.x < a.np) dem_particle(a, threadIdx.x);
        __syncthreads();
    }
}

// Up to DEM_LDS particles: as k_dem_one_wg, with the particle state kept in
// LDS through the sub-steps (two copies in place of the two global buffers),
// so that a sub-step reads its own and its neighbours' states without a
// round trip to L2.  Both copies go back to the global buffers at the end:
// these then hold what the sub-steps one launch each would leave.
constexpr int DEM_LDS = 256;
__global__ __launch_bounds__(DEM_LDS) void k_dem_one_wg_lds(DemOneWg f)
{
    __shared__ DevParticle buf[2][DEM_LDS];
    const int i = threadIdx.x;
    const bool mine = i < f.a.np;
    if (mine) buf[0][i] = f.part[0][i];
    __syncthreads();
    for (int s = 0; s < f.n_sub; ++s) {
        DemArgs a = f.a;
        const int c = s & 1;
        a.cur = buf[c];
        a.nxt = buf[c ^ 1];
        a.hid_in = f.hid[c]; a.hxi_in = f.hxi[c]; a.hn_in = f.hn[c];
        a.hid_out = f.hid[c ^ 1]; a.hxi_out = f.hxi[c ^ 1]; a.hn_out = f.hn[c ^ 1];
        a.last = s == f.n_sub - 1;
        if (mine) dem_particle(a, i);
        __syncthreads();
    }
    if (mine) {
        f.part[0][i] = buf[0][i];
        if (f.n_sub > 0) f.part[1][i] = buf[1][i];
    }
}


// Initial state: f = w rho0 and g = w T_init, i.e. deviations 0 and
// w (T_init - T_s) (dTinit), T_s the temperature the g deviations are stored from.
template <class SF, class L>
__global__ void k_init(void *f, void *g, long long N, long long Ns, typename SF::T dTinit)
{
    using S = typename SF::S;
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
        for (int q = 0; q < L::Q; ++q) SF::st((S *)f + (size_t)q * Ns + n, (typename SF::T)0, 1.0);
        for (int q = 0; q < L::QG; ++q)
            SF::st((S *)g + (size_t)q * Ns + n, (typename SF::T)(L::wg(q) * (double)dTinit), L::wg(q));
    }
}

}  // namespace pibm
