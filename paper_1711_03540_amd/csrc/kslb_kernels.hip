// kslb_kernels.hip -- gfx950 kernels of the KS lattice Boltzmann scheme.
//
// One LB step (paper section 2, Eq. (2)) in pull form on post-collision
// populations S:
//     g_i(j)  = S_i(j - c_i)                       (streaming)
//     rho_j   = sum_i g_i(j)                        (density, fixed order)
//     S'_i(j) = (1 - omega) g_i + omega feq_i(rho_j),  feq_i = E_i rho + G_i rho^2
// Every kernel class below evaluates that step through the same inline
// functions (Pol<Q,P>::pop and Pol<Q,P>::update) with explicit FMAs and
// -ffp-contract=off, so the plain, ring and tiled kernels and the ensemble
// kernel produce bitwise identical states.
//
// Layout in HBM: structure of arrays, population-major, one copy per
// ping-pong side, rows padded to a pitch p = n rounded up to 64 sites.
// FP64: Q rows of p doubles.  FP32: Q rows of p floats.  SPLIT: one row of p
// doubles (rho), then Q rows of p floats (f_i - feq_i(rho)).
//
// Register-resident kernels give each lane B consecutive sites in VGPRs.  A
// step moves data between lanes only at block edges: lane l publishes the
// populations its neighbours pull (the last c sites of each c > 0 population,
// the first |c| of each c < 0 one; 12 doubles for D1Q7, 6 for D1Q5) to a
// double-buffered LDS exchange area, one barrier, then every site is updated
// from registers plus the neighbours' values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <utility>

#include "kslb_internal.h"

namespace kslb {

// ---------------------------------------------------------------- lattice constants

__host__ __device__ constexpr int vel(int i) { return i == 0 ? 0 : ((i & 1) ? (i + 1) / 2 : -(i / 2)); }
__host__ __device__ constexpr int iabs(int v) { return v < 0 ? -v : v; }
__host__ __device__ constexpr int halo_of(int q) { return q == 5 ? 2 : 3; }
// G_i = J w1_i is nonzero only for c = +-1, +-2
__host__ __device__ constexpr bool has_g(int i) { return i >= 1 && i <= 4; }
// halo values exchanged per lane per step, and offset of population i in them
__host__ __device__ constexpr int nx_of(int q) { return q == 5 ? 6 : 12; }
__host__ __device__ constexpr int koff(int i)
{
    int k = 0;
    for (int a = 1; a < i; a++) k += iabs(vel(a));
    return k;
}

template <int... Is, class F>
__device__ __forceinline__ void unroll_impl(std::integer_sequence<int, Is...>, F&& f)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll(F&& f)
{
    unroll_impl(std::make_integer_sequence<int, N>{}, f);
}

__device__ __forceinline__ int64_t wrap_site(int64_t j, int64_t n)
{
    j %= n;
    return j < 0 ? j + n : j;
}

// Density sum over the incoming populations in a fixed pairwise order (every
// kernel class uses this one, so they round identically).
template <int Q>
__device__ __forceinline__ double dsum(const double (&g)[Q])
{
    if constexpr (Q == 5) return ((g[0] + g[1]) + (g[2] + g[3])) + g[4];
    else return ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + g[6]);
}

// Equilibrium feq_i(rho) = e_i rho + g_i rho^2 with (e, g) = (E, G) or, with
// omega folded in, (A, B) = omega (E, G).  The equilibrium of Eq. (feq) is
// built from the even-moment weights w(0), w(2), w(4) (and w(6) for D1Q7),
// which take equal values at +c and -c, and from the first-moment weight w(1),
// which changes sign; so e_{+c} = e_{-c} and g_{+c} = -g_{-c} exactly, and a
// +-c pair shares its product e rho.  eq_one and eq_all round identically.
// eq_one takes e of the pair's +c member, so that the two members evaluated
// from one density share the product e rho
template <int I>
__device__ __forceinline__ double eq_one(double rho, const double* e, const double* g)
{
    constexpr int ie = (I > 0 && I % 2 == 0) ? I - 1 : I;
    if constexpr (has_g(I)) return __builtin_fma(g[I], rho * rho, e[ie] * rho);
    else return e[ie] * rho;
}

template <int Q>
__device__ __forceinline__ void eq_all(double rho, const double* e, const double* g, double (&eq)[Q])
{
    const double r2 = rho * rho;
    eq[0] = e[0] * rho;
    unroll<(Q - 1) / 2>([&](auto K) {
        constexpr int ip = 2 * K + 1, im = 2 * K + 2;   // velocities +c, -c
        const double a = e[ip] * rho;
        if constexpr (has_g(ip)) {
            eq[ip] = __builtin_fma(g[ip], r2, a);
            eq[im] = __builtin_fma(g[im], r2, a);
        } else {
            eq[ip] = a;
            eq[im] = a;
        }
    });
}

typedef double d2v __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- precision policies
// A state copy stores population i of site j at element i * p + j, with the
// row pitch p = n rounded up to a multiple of 64 (see state_pitch).

template <int Q, int P>
struct Pol;

template <int Q>
struct Pol<Q, kFP64> {
    struct Site { double s[Q]; };

    template <int I>
    __device__ static __forceinline__ double pop(const Site& x, const Coef&) { return x.s[I]; }

    template <int I>
    __device__ static __forceinline__ double pop_g(const char* st, int64_t p, int64_t j, const Coef&)
    {
        return reinterpret_cast<const double*>(st)[I * p + j];
    }

    __device__ static __forceinline__ void update(const double (&g)[Q], Site& y, const Coef& cf)
    {
        double eq[Q];
        eq_all<Q>(dsum<Q>(g), cf.A, cf.B, eq);
        unroll<Q>([&](auto I) { y.s[I] = __builtin_fma(cf.a1mw, g[I], eq[I]); });
    }

    __device__ static __forceinline__ Site load(const char* st, int64_t p, int64_t j)
    {
        Site x;
        unroll<Q>([&](auto I) { x.s[I] = reinterpret_cast<const double*>(st)[I * p + j]; });
        return x;
    }

    __device__ static __forceinline__ void store(char* st, int64_t p, int64_t j, const Site& x)
    {
        unroll<Q>([&](auto I) { reinterpret_cast<double*>(st)[I * p + j] = x.s[I]; });
    }

    // as store, with non-temporal hints (streaming writes no later access in
    // the same launch reads)
    __device__ static __forceinline__ void store_nt(char* st, int64_t p, int64_t j, const Site& x)
    {
        unroll<Q>([&](auto I) { __builtin_nontemporal_store(x.s[I], reinterpret_cast<double*>(st) + I * p + j); });
    }

    // B consecutive sites from j0 (j0 and p multiples of 2)
    template <int B>
    __device__ static __forceinline__ void load_vec(const char* st, int64_t p, int64_t j0, Site (&x)[B])
    {
        unroll<Q>([&](auto I) {
            const d2v* src = reinterpret_cast<const d2v*>(reinterpret_cast<const double*>(st) + I * p + j0);
            unroll<B / 2>([&](auto K) {
                const d2v v = src[K];
                x[2 * K].s[I] = v.x;
                x[2 * K + 1].s[I] = v.y;
            });
        });
    }

    template <int B>
    __device__ static __forceinline__ void store_vec(char* st, int64_t p, int64_t j0, const Site (&x)[B])
    {
        unroll<Q>([&](auto I) {
            d2v* dst = reinterpret_cast<d2v*>(reinterpret_cast<double*>(st) + I * p + j0);
            unroll<B / 2>([&](auto K) {
                d2v v;
                v.x = x[2 * K].s[I];
                v.y = x[2 * K + 1].s[I];
                dst[K] = v;
            });
        });
    }

    __device__ static __forceinline__ Site equilibrium(double rho, const Coef& cf)
    {
        Site x;
        eq_all<Q>(rho, cf.E, cf.G, x.s);
        return x;
    }

    __device__ static __forceinline__ Site from_f(const double (&f)[Q], const Coef&)
    {
        Site x;
        unroll<Q>([&](auto I) { x.s[I] = f[I]; });
        return x;
    }

    __device__ static __forceinline__ double density(const Site& x) { return dsum<Q>(x.s); }

    __device__ static __forceinline__ bool finite(const Site& x)
    {
        bool ok = true;
        unroll<Q>([&](auto I) { ok = ok && __builtin_isfinite(x.s[I]); });
        return ok;
    }
};

template <int Q>
struct Pol<Q, kFP32> {
    struct Site { float s[Q]; };

    template <int I>
    __device__ static __forceinline__ double pop(const Site& x, const Coef&) { return (double)x.s[I]; }

    template <int I>
    __device__ static __forceinline__ double pop_g(const char* st, int64_t p, int64_t j, const Coef&)
    {
        return (double)reinterpret_cast<const float*>(st)[I * p + j];
    }

    // density sum and rho^2 term in double, relaxation in single
    __device__ static __forceinline__ void update(const double (&g)[Q], Site& y, const Coef& cf)
    {
        double eq[Q];
        eq_all<Q>(dsum<Q>(g), cf.A, cf.B, eq);
        unroll<Q>([&](auto I) { y.s[I] = __builtin_fmaf(cf.a1mw_f, (float)g[I], (float)eq[I]); });
    }

    __device__ static __forceinline__ Site load(const char* st, int64_t p, int64_t j)
    {
        Site x;
        unroll<Q>([&](auto I) { x.s[I] = reinterpret_cast<const float*>(st)[I * p + j]; });
        return x;
    }

    __device__ static __forceinline__ void store(char* st, int64_t p, int64_t j, const Site& x)
    {
        unroll<Q>([&](auto I) { reinterpret_cast<float*>(st)[I * p + j] = x.s[I]; });
    }

    __device__ static __forceinline__ void store_nt(char* st, int64_t p, int64_t j, const Site& x)
    {
        unroll<Q>([&](auto I) { __builtin_nontemporal_store(x.s[I], reinterpret_cast<float*>(st) + I * p + j); });
    }

    // B consecutive sites from j0 (B and j0 even): 8-byte accesses, two sites
    // of one population each
    template <int B>
    __device__ static __forceinline__ void load_vec(const char* st, int64_t p, int64_t j0, Site (&x)[B])
    {
        unroll<Q>([&](auto I) {
            const uint64_t* src = reinterpret_cast<const uint64_t*>(reinterpret_cast<const float*>(st) + I * p + j0);
            unroll<B / 2>([&](auto K) {
                const uint64_t v = src[K];
                x[2 * K].s[I] = __uint_as_float((unsigned)v);
                x[2 * K + 1].s[I] = __uint_as_float((unsigned)(v >> 32));
            });
        });
    }

    template <int B>
    __device__ static __forceinline__ void store_vec(char* st, int64_t p, int64_t j0, const Site (&x)[B])
    {
        unroll<Q>([&](auto I) {
            uint64_t* dst = reinterpret_cast<uint64_t*>(reinterpret_cast<float*>(st) + I * p + j0);
            unroll<B / 2>([&](auto K) {
                dst[K] = (uint64_t)__float_as_uint(x[2 * K].s[I]) |
                         ((uint64_t)__float_as_uint(x[2 * K + 1].s[I]) << 32);
            });
        });
    }

    __device__ static __forceinline__ Site equilibrium(double rho, const Coef& cf)
    {
        Site x;
        double eq[Q];
        eq_all<Q>(rho, cf.E, cf.G, eq);
        unroll<Q>([&](auto I) { x.s[I] = (float)eq[I]; });
        return x;
    }

    __device__ static __forceinline__ Site from_f(const double (&f)[Q], const Coef&)
    {
        Site x;
        unroll<Q>([&](auto I) { x.s[I] = (float)f[I]; });
        return x;
    }

    __device__ static __forceinline__ double density(const Site& x)
    {
        double g[Q];
        unroll<Q>([&](auto I) { g[I] = (double)x.s[I]; });
        return dsum<Q>(g);
    }

    __device__ static __forceinline__ bool finite(const Site& x)
    {
        bool ok = true;
        unroll<Q>([&](auto I) { ok = ok && __builtin_isfinite(x.s[I]); });
        return ok;
    }
};

// rho in double, non-equilibrium part n_i = S_i - feq_i(rho) in single.
// Copy layout: one row of p doubles (rho), then Q rows of p floats.
template <int Q>
struct Pol<Q, kSPLIT> {
    struct Site { double rho; float n[Q]; };

    __device__ static __forceinline__ const float* nbase(const char* st, int64_t p)
    {
        return reinterpret_cast<const float*>(st + p * (int64_t)sizeof(double));
    }

    template <int I>
    __device__ static __forceinline__ double eq_of(double rho, const Coef& cf)
    {
        return eq_one<I>(rho, cf.E, cf.G);
    }

    template <int I>
    __device__ static __forceinline__ double pop(const Site& x, const Coef& cf)
    {
        return eq_of<I>(x.rho, cf) + (double)x.n[I];
    }

    template <int I>
    __device__ static __forceinline__ double pop_g(const char* st, int64_t p, int64_t j, const Coef& cf)
    {
        const double rho = reinterpret_cast<const double*>(st)[j];
        return eq_of<I>(rho, cf) + (double)nbase(st, p)[I * p + j];
    }

    __device__ static __forceinline__ void update(const double (&g)[Q], Site& y, const Coef& cf)
    {
        const double rho = dsum<Q>(g);
        y.rho = rho;
        double eq[Q];
        eq_all<Q>(rho, cf.E, cf.G, eq);
        unroll<Q>([&](auto I) { y.n[I] = (float)(cf.a1mw * (g[I] - eq[I])); });
    }

    __device__ static __forceinline__ Site load(const char* st, int64_t p, int64_t j)
    {
        Site x;
        x.rho = reinterpret_cast<const double*>(st)[j];
        const float* nb = nbase(st, p);
        unroll<Q>([&](auto I) { x.n[I] = nb[I * p + j]; });
        return x;
    }

    __device__ static __forceinline__ void store(char* st, int64_t p, int64_t j, const Site& x)
    {
        reinterpret_cast<double*>(st)[j] = x.rho;
        float* nb = const_cast<float*>(nbase(st, p));
        unroll<Q>([&](auto I) { nb[I * p + j] = x.n[I]; });
    }

    __device__ static __forceinline__ void store_nt(char* st, int64_t p, int64_t j, const Site& x)
    {
        __builtin_nontemporal_store(x.rho, reinterpret_cast<double*>(st) + j);
        float* nb = const_cast<float*>(nbase(st, p));
        unroll<Q>([&](auto I) { __builtin_nontemporal_store(x.n[I], nb + I * p + j); });
    }

    // B consecutive sites from j0 (B and j0 even): 16-byte density and
    // 8-byte non-equilibrium accesses
    template <int B>
    __device__ static __forceinline__ void load_vec(const char* st, int64_t p, int64_t j0, Site (&x)[B])
    {
        const d2v* r = reinterpret_cast<const d2v*>(reinterpret_cast<const double*>(st) + j0);
        unroll<B / 2>([&](auto K) {
            const d2v v = r[K];
            x[2 * K].rho = v.x;
            x[2 * K + 1].rho = v.y;
        });
        unroll<Q>([&](auto I) {
            const uint64_t* src = reinterpret_cast<const uint64_t*>(nbase(st, p) + I * p + j0);
            unroll<B / 2>([&](auto K) {
                const uint64_t v = src[K];
                x[2 * K].n[I] = __uint_as_float((unsigned)v);
                x[2 * K + 1].n[I] = __uint_as_float((unsigned)(v >> 32));
            });
        });
    }

    template <int B>
    __device__ static __forceinline__ void store_vec(char* st, int64_t p, int64_t j0, const Site (&x)[B])
    {
        d2v* r = reinterpret_cast<d2v*>(reinterpret_cast<double*>(st) + j0);
        unroll<B / 2>([&](auto K) {
            d2v v;
            v.x = x[2 * K].rho;
            v.y = x[2 * K + 1].rho;
            r[K] = v;
        });
        unroll<Q>([&](auto I) {
            uint64_t* dst = reinterpret_cast<uint64_t*>(const_cast<float*>(nbase(st, p)) + I * p + j0);
            unroll<B / 2>([&](auto K) {
                dst[K] = (uint64_t)__float_as_uint(x[2 * K].n[I]) |
                         ((uint64_t)__float_as_uint(x[2 * K + 1].n[I]) << 32);
            });
        });
    }

    __device__ static __forceinline__ Site equilibrium(double rho, const Coef&)
    {
        Site x;
        x.rho = rho;
        unroll<Q>([&](auto I) { x.n[I] = 0.0f; });
        return x;
    }

    __device__ static __forceinline__ Site from_f(const double (&f)[Q], const Coef& cf)
    {
        Site x;
        const double rho = dsum<Q>(f);
        x.rho = rho;
        unroll<Q>([&](auto I) { x.n[I] = (float)(f[I] - eq_of<I>(rho, cf)); });
        return x;
    }

    __device__ static __forceinline__ double density(const Site& x) { return x.rho; }

    __device__ static __forceinline__ bool finite(const Site& x)
    {
        bool ok = __builtin_isfinite(x.rho);
        unroll<Q>([&](auto I) { ok = ok && __builtin_isfinite(x.n[I]); });
        return ok;
    }
};

// tau = 1 only (omega = 1): the collision leaves S_i = feq_i(rho), so the
// state is rho alone, one row of p doubles.  A population is rebuilt as
// feq_i(rho) by the same expression the FP64 policy evaluates with
// A_i = 1 * E_i and B_i = 1 * G_i, so densities are bitwise those of FP64.
template <int Q>
struct Pol<Q, kRHO> {
    struct Site { double rho; };

    template <int I>
    __device__ static __forceinline__ double eq_of(double rho, const Coef& cf)
    {
        return eq_one<I>(rho, cf.A, cf.B);
    }

    template <int I>
    __device__ static __forceinline__ double pop(const Site& x, const Coef& cf) { return eq_of<I>(x.rho, cf); }

    template <int I>
    __device__ static __forceinline__ double pop_g(const char* st, int64_t, int64_t j, const Coef& cf)
    {
        return eq_of<I>(reinterpret_cast<const double*>(st)[j], cf);
    }

    __device__ static __forceinline__ void update(const double (&g)[Q], Site& y, const Coef&)
    {
        y.rho = dsum<Q>(g);
    }

    __device__ static __forceinline__ Site load(const char* st, int64_t, int64_t j)
    {
        return Site{reinterpret_cast<const double*>(st)[j]};
    }

    __device__ static __forceinline__ void store(char* st, int64_t, int64_t j, const Site& x)
    {
        reinterpret_cast<double*>(st)[j] = x.rho;
    }

    // plain stores here: with one double per site the non-temporal hint
    // measured slower (227 against 296 GLUPS, D1Q7 at N = 2^24)
    __device__ static __forceinline__ void store_nt(char* st, int64_t p, int64_t j, const Site& x) { store(st, p, j, x); }

    template <int B>
    __device__ static __forceinline__ void load_vec(const char* st, int64_t, int64_t j0, Site (&x)[B])
    {
        const d2v* r = reinterpret_cast<const d2v*>(reinterpret_cast<const double*>(st) + j0);
        unroll<B / 2>([&](auto K) {
            const d2v v = r[K];
            x[2 * K].rho = v.x;
            x[2 * K + 1].rho = v.y;
        });
    }

    template <int B>
    __device__ static __forceinline__ void store_vec(char* st, int64_t, int64_t j0, const Site (&x)[B])
    {
        d2v* r = reinterpret_cast<d2v*>(reinterpret_cast<double*>(st) + j0);
        unroll<B / 2>([&](auto K) {
            d2v v;
            v.x = x[2 * K].rho;
            v.y = x[2 * K + 1].rho;
            r[K] = v;
        });
    }

    __device__ static __forceinline__ Site equilibrium(double rho, const Coef&) { return Site{rho}; }

    __device__ static __forceinline__ Site from_f(const double (&f)[Q], const Coef&) { return Site{dsum<Q>(f)}; }

    __device__ static __forceinline__ double density(const Site& x) { return x.rho; }

    __device__ static __forceinline__ bool finite(const Site& x) { return __builtin_isfinite(x.rho); }
};

// ---------------------------------------------------------------- per-site kernels

template <int Q, int P>
__global__ __launch_bounds__(256) void k_init(char* st, int64_t n, int64_t p, const double* __restrict__ rho0,
                                              Coef cf)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) PL::store(st, p, j, PL::equilibrium(rho0[j], cf));
}

// Equilibrium init of many lattices in one launch: block row y initialises
// instance d[y] (its descriptor and coefficient set are uniform over the
// block), block column x its sites [256 x, 256 x + 256).
template <int Q, int P>
__global__ __launch_bounds__(256) void k_init_many(const InstDesc* __restrict__ d,
                                                   const Coef* __restrict__ coefs, const double* __restrict__ rho)
{
    using PL = Pol<Q, P>;
    const InstDesc e = d[blockIdx.y];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < e.n)
        PL::store(reinterpret_cast<char*>(e.state), e.pitch, j, PL::equilibrium(rho[e.rho_off + j], coefs[e.coef]));
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Renumber them so that XCD x runs a contiguous run of logical blocks: the
// halo lines two neighbouring tiles share then sit in one L2.  Used by the
// tiled kernel only: the one-step streaming kernel reads each line once and
// runs faster in hardware order (49.8 against 47.6 GLUPS at N = 2^24, D1Q7,
// FP64, measured back to back), where all eight XCDs stream neighbouring
// addresses at the same time.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t per = nb / 8;
    if (b < per * 8) return (b % 8) * per + b / 8;
    return b;   // the ragged remainder keeps its index
}

// One fused pull-stream + density + equilibrium + BGK step per launch (s = 1).
template <int Q, int P>
__global__ __launch_bounds__(256) void k_plain(const char* __restrict__ src, char* __restrict__ dst,
                                               int64_t n, int64_t p, Coef cf)
{
    using PL = Pol<Q, P>;
    constexpr int H = halo_of(Q);
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double g[Q];
    if (j >= H && j + H < n) {
        unroll<Q>([&](auto I) { g[I] = PL::template pop_g<I>(src, p, j - vel(I), cf); });
    } else {
        unroll<Q>([&](auto I) { g[I] = PL::template pop_g<I>(src, p, wrap_site(j - vel(I), n), cf); });
    }
    typename PL::Site y;
    PL::update(g, y, cf);
    // non-temporal stores (except for the rho-only state): at N = 2^24, D1Q7
    // FP64 streams 5.70 TB/s against 5.58 with plain stores, FP32 and split
    // gain 4 %, D1Q5 3-4 % (bitwise the same state)
    PL::store_nt(dst, p, j, y);
}

// Fixed ends (the Table 3 problem of section 3): sites 0 and n-1 and the
// ghosts beyond them hold the end-value equilibria; a streamed population
// from beyond an end is that end's equilibrium value.
template <int Q, int P>
__global__ __launch_bounds__(256) void k_plain_fixed(const char* __restrict__ src, char* __restrict__ dst,
                                                     int64_t n, int64_t p, Coef cf, double rho_l, double rho_r)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    if (j == 0 || j == n - 1) {
        PL::store(dst, p, j, PL::equilibrium(j == 0 ? rho_l : rho_r, cf));
        return;
    }
    const auto eq_l = PL::equilibrium(rho_l, cf), eq_r = PL::equilibrium(rho_r, cf);
    double g[Q];
    unroll<Q>([&](auto I) {
        const int64_t sj = j - vel(I);
        if (sj < 0) g[I] = PL::template pop<I>(eq_l, cf);
        else if (sj >= n) g[I] = PL::template pop<I>(eq_r, cf);
        else g[I] = PL::template pop_g<I>(src, p, sj, cf);
    });
    typename PL::Site y;
    PL::update(g, y, cf);
    PL::store(dst, p, j, y);
}

template <int Q, int P>
__global__ __launch_bounds__(256) void k_init_fixed(char* st, int64_t n, int64_t p, const double* __restrict__ rho0,
                                                    Coef cf, double rho_l, double rho_r)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) PL::store(st, p, j, PL::equilibrium(j == 0 ? rho_l : (j == n - 1 ? rho_r : rho0[j]), cf));
}

// ---------------------------------------------------------------- register-resident step engine

// LD = lanes stride of the exchange area (compile time, so every LDS address
// is the lane's base plus an immediate offset).
template <int Q, int P, int B, int LD>
struct Engine {
    using PL = Pol<Q, P>;
    using Site = typename PL::Site;
    static constexpr int H = halo_of(Q);
    // rho-only state: the neighbours need the densities of the H edge sites
    // on each side, not the 12 (6) populations
    static constexpr bool kR = (P == kRHO);

    // Where site b of this lane streams population i from: site sb = b - c_i
    // in this lane's numbering, i.e. site rem_site(i, b) of the lane
    // rem_lane(i, b) lanes away (negative: to the left).  With at least max|c|
    // sites per lane every remote source is a neighbouring lane; single-wave
    // engines also take fewer, with sources up to ceil(max|c| / B) lanes away.
    static constexpr int sdiv(int a) { return a >= 0 ? a / B : -((-a + B - 1) / B); }
    static constexpr bool is_remote(int i, int b) { return b - vel(i) < 0 || b - vel(i) >= B; }
    static constexpr int rem_lane(int i, int b) { return sdiv(b - vel(i)); }
    static constexpr int rem_site(int i, int b) { return (b - vel(i)) - rem_lane(i, b) * B; }
    // index of the remote value (i, b) among all remote values, population by
    // population and site by site; with B >= max|c| this is koff(i) plus the
    // value's place in its population, the layout the LDS exchange writes
    static constexpr int rslot(int i, int b)
    {
        int k = 0;
        for (int i2 = 0; i2 < Q; i2++)
            for (int b2 = 0; b2 < B; b2++) {
                if (i2 == i && b2 == b) return k;
                if (is_remote(i2, b2)) k++;
            }
        return k;
    }
    static constexpr int NR = rslot(Q, 0);   // remote values per lane and step
    static constexpr int NX = kR ? 2 * H : NR;
    static constexpr int SLOT = NX * LD;     // exchanged values per buffer
    static_assert(B >= H || (LD == 64 && !kR),
                  "a lane holds at least max|c| sites, except in single-wave engines of populations");
    static_assert(B < H || kR || NR == nx_of(Q), "neighbour exchange layout");
    // Exchanged value: FP32 populations travel as stored (widening them to
    // double is exact, so the receiver widens them instead); every other
    // state sends the double population (or density) its update reads.
    static constexpr bool kF = (P == kFP32);
    using XV = typename std::conditional<kF, float, double>::type;
    template <int i>
    __device__ static __forceinline__ XV xval(const Site& s, const Coef& cf)
    {
        if constexpr (kF) return s.s[i];
        else return PL::template pop<i>(s, cf);
    }

    // write the values the neighbours pull (column `lane` of slot)
    __device__ static __forceinline__ void publish(const Site (&x)[B], XV* slot, const Coef& cf)
    {
        if constexpr (kR) {
            unroll<H>([&](auto T) {
                slot[T * LD] = x[B - H + T].rho;           // for the right neighbour
                slot[(H + T) * LD] = x[T].rho;             // for the left neighbour
            });
        } else {
            unroll<Q - 1>([&](auto I1) {
                constexpr int i = I1 + 1;
                constexpr int c = vel(i);
                constexpr int k0 = koff(i);
                unroll<iabs(c)>([&](auto T) {
                    constexpr int t = T;
                    constexpr int src = (c > 0) ? (B - c + t) : t;
                    slot[(k0 + t) * LD] = xval<i>(x[src], cf);
                });
            });
        }
    }

    // one step x -> y from registers plus hv, the values pulled from the
    // neighbour lanes (hv[koff(i) + t] as published by publish_vals)
    // sites whose sources all lie in this lane (H <= b < B - H) first, so the
    // neighbours' values have time to arrive; then the edge sites
    template <bool INTERIOR>
    __device__ static __forceinline__ void step_sites(const Site (&x)[B], Site (&y)[B], const XV (&hv)[NX],
                                                      const Coef& cf)
    {
        unroll<B>([&](auto Bi) {
            constexpr int b = Bi;
            if constexpr ((b >= H && b < B - H) != INTERIOR) return;
            double g[Q];
            unroll<Q>([&](auto I) {
                constexpr int i = I;
                constexpr int c = vel(i);
                constexpr int sb = b - c;
                if constexpr (sb >= 0 && sb < B) g[i] = PL::template pop<i>(x[sb], cf);
                else if constexpr (kR) g[i] = PL::template pop<i>(Site{hv[sb < 0 ? H + sb : H + sb - B]}, cf);
                else g[i] = (double)hv[rslot(i, b)];
            });
            PL::update(g, y[b], cf);
        });
    }

    __device__ static __forceinline__ void step_hv(const Site (&x)[B], Site (&y)[B], const XV (&hv)[NX],
                                                   const Coef& cf)
    {
        step_sites<true>(x, y, hv, cf);
        step_sites<false>(x, y, hv, cf);
    }

    // one step x -> y: left/right point at the neighbours' columns of the slot
    __device__ static __forceinline__ void step(const Site (&x)[B], Site (&y)[B], const XV* left,
                                                const XV* right, const Coef& cf)
    {
        XV hv[NX];
        if constexpr (kR) {
            unroll<H>([&](auto T) {
                hv[T] = left[T * LD];
                hv[H + T] = right[(H + T) * LD];
            });
        } else {
            unroll<Q - 1>([&](auto I1) {
                constexpr int i = I1 + 1;
                constexpr int c = vel(i);
                constexpr int k0 = koff(i);
                unroll<iabs(c)>([&](auto T) {
                    constexpr int t = T;
                    hv[k0 + t] = (c > 0 ? left : right)[(k0 + t) * LD];
                });
            });
        }
        step_hv(x, y, hv, cf);
    }

    // One step x -> y that computes and publishes the edge sites first (out:
    // this lane's column of the other exchange buffer), at raised wave
    // priority, then the interior: the values the neighbours wait for at the
    // next barrier leave as early as possible.  (Without the priority change,
    // which also bounds the compiler's reordering, the same order measured
    // slower for D1Q7 FP64; with it D1Q7 FP64 is unchanged, D1Q5 FP64 and
    // FP32 run 3-4 % faster.)
    __device__ static __forceinline__ void step_ep(const Site (&x)[B], Site (&y)[B], const XV* left,
                                                   const XV* right, XV* out, const Coef& cf)
    {
        XV hv[NX];
        if constexpr (kR) {
            unroll<H>([&](auto T) {
                hv[T] = left[T * LD];
                hv[H + T] = right[(H + T) * LD];
            });
        } else {
            unroll<Q - 1>([&](auto I1) {
                constexpr int i = I1 + 1;
                constexpr int c = vel(i);
                constexpr int k0 = koff(i);
                unroll<iabs(c)>([&](auto T) {
                    constexpr int t = T;
                    hv[k0 + t] = (c > 0 ? left : right)[(k0 + t) * LD];
                });
            });
        }
        __builtin_amdgcn_s_setprio(1);
        step_sites<false>(x, y, hv, cf);
        publish(y, out, cf);
        __builtin_amdgcn_s_setprio(0);
        step_sites<true>(x, y, hv, cf);
    }

    // Single-wave windows: the neighbour values move between lanes with DPP
    // wave rotations (lane l reads lane l-1 for c > 0, lane l+1 for c < 0),
    // with no LDS round trip and no barrier.
    // A whole-wave rotation gives every lane a valid source lane, so the
    // destination's previous value is never kept and need not be set first.
    __device__ static __forceinline__ double from_lane(double v, bool from_left)
    {
        const int lo = __double2loint(v), hi = __double2hiint(v);
        int rlo, rhi;
        if (from_left) {
            rlo = __builtin_amdgcn_mov_dpp(lo, 0x13C, 0xF, 0xF, true);   // wave_ror:1
            rhi = __builtin_amdgcn_mov_dpp(hi, 0x13C, 0xF, 0xF, true);
        } else {
            rlo = __builtin_amdgcn_mov_dpp(lo, 0x134, 0xF, 0xF, true);   // wave_rol:1
            rhi = __builtin_amdgcn_mov_dpp(hi, 0x134, 0xF, 0xF, true);
        }
        return __hiloint2double(rhi, rlo);
    }
    __device__ static __forceinline__ float from_lane(float v, bool from_left)
    {
        const int u = __float_as_int(v);
        return __int_as_float(from_left ? __builtin_amdgcn_mov_dpp(u, 0x13C, 0xF, 0xF, true)     // wave_ror:1
                                        : __builtin_amdgcn_mov_dpp(u, 0x134, 0xF, 0xF, true));   // wave_rol:1
    }

    __device__ static __forceinline__ void step_dpp(const Site (&x)[B], Site (&y)[B], const Coef& cf)
    {
        XV hv[NX];
        if constexpr (kR) {
            unroll<H>([&](auto T) {
                hv[T] = from_lane(x[B - H + T].rho, true);
                hv[H + T] = from_lane(x[T].rho, false);
            });
        } else {
            // each remote value moves |rem_lane| lanes, one rotation per lane
            unroll<Q>([&](auto I) {
                unroll<B>([&](auto Bi) {
                    constexpr int i = I, b = Bi;
                    if constexpr (is_remote(i, b)) {
                        constexpr int d = rem_lane(i, b);
                        XV v = xval<i>(x[rem_site(i, b)], cf);
                        unroll<iabs(d)>([&](auto) { v = from_lane(v, d < 0); });
                        hv[rslot(i, b)] = v;
                    }
                });
            });
        }
        step_hv(x, y, hv, cf);
    }

    // `steps` steps in place on x, lanes `lane` with neighbour lanes left/right;
    // every lane of the workgroup must call this (it holds the barriers).
    struct NoFix {
        __device__ __forceinline__ void operator()(Site (&)[B]) const {}
    };

    // fix(x) runs after every step (the fixed-end boundary of section 3's
    // Table 3 problem re-imposes its end states there); NoFix for periodic.
    template <class Fix = NoFix>
    __device__ static __forceinline__ void run(Site (&x)[B], int64_t steps, double* xch, int lane, int left,
                                               int right, bool active, const Coef& cf, const Fix& fix = Fix())
    {
        Site y[B];
        int64_t st = 0;
        if constexpr (LD == 64) {
            // one wave: lanes are neighbours modulo 64, exchange by DPP
            (void)xch; (void)lane; (void)left; (void)right; (void)active;
            for (; st + 1 < steps; st += 2) {
                step_dpp(x, y, cf);
                fix(y);
                step_dpp(y, x, cf);
                fix(x);
            }
            if (st < steps) {
                step_dpp(x, y, cf);
                unroll<B>([&](auto Bi) { x[Bi] = y[Bi]; });
                fix(x);
            }
        } else {
            XV* xb = reinterpret_cast<XV*>(xch);   // the exchange area, in exchanged values
            if constexpr (std::is_same<Fix, NoFix>::value) {
                // each step publishes its own edges into the buffer the next
                // step reads: one barrier per step, buffers alternating
                if (active) publish(x, xb + lane, cf);
                __syncthreads();
                for (; st + 1 < steps; st += 2) {
                    if (active) step_ep(x, y, xb + left, xb + right, xb + SLOT + lane, cf);
                    __syncthreads();
                    if (active) step_ep(y, x, xb + SLOT + left, xb + SLOT + right, xb + lane, cf);
                    __syncthreads();
                }
                if (st < steps) {
                    if (active) {
                        step(x, y, xb + left, xb + right, cf);
                        unroll<B>([&](auto Bi) { x[Bi] = y[Bi]; });
                    }
                    __syncthreads();   // the next call writes slot 0 again
                }
                return;
            }
            for (; st + 1 < steps; st += 2) {
                if (active) publish(x, xb + lane, cf);
                __syncthreads();
                if (active) {
                    step(x, y, xb + left, xb + right, cf);
                    fix(y);
                    publish(y, xb + SLOT + lane, cf);
                }
                __syncthreads();
                if (active) {
                    step(y, x, xb + SLOT + left, xb + SLOT + right, cf);
                    fix(x);
                }
            }
            if (st < steps) {
                if (active) publish(x, xb + lane, cf);
                __syncthreads();
                if (active) {
                    step(x, y, xb + left, xb + right, cf);
                    unroll<B>([&](auto Bi) { x[Bi] = y[Bi]; });
                    fix(x);
                }
                __syncthreads();   // the next call writes slot 0 again
            }
        }
    }
};

constexpr int kRingLD = 512;

constexpr int kTileLD = 256;

// Whole periodic lattice of n = B * L sites in one workgroup of L lanes,
// `steps` steps per launch; lane 0 and lane L-1 are neighbours.
template <int Q, int P, int B>
__global__ __launch_bounds__(kRingLD) void k_ring(const char* __restrict__ src, char* __restrict__ dst,
                                                  int n, int64_t p, int64_t steps, Coef cf)
{
    using E = Engine<Q, P, B, kRingLD>;
    extern __shared__ double xch[];
    const int L = n / B;
    const int lane = threadIdx.x;
    const bool active = lane < L;
    typename E::Site x[B];
    if (active) E::PL::template load_vec<B>(src, p, (int64_t)lane * B, x);
    const int left = lane == 0 ? L - 1 : lane - 1;
    const int right = lane + 1 >= L ? 0 : lane + 1;
    E::run(x, steps, xch, lane, left, right, active, cf);
    if (active) E::PL::template store_vec<B>(dst, p, (int64_t)lane * B, x);
}

// One lane's part of a halo-widened window.  The lane holds sites j0 .. j0+B-1
// of a periodic lattice of n sites (taken modulo n), which are slots
// kl0 .. kl0+B-1 of its segment; after s steps the slots [k_lo, k_lo + valid)
// of the segment are exact and are written back (slots near a segment's
// ends go stale by H per step and are never stored).  Every lane of the
// workgroup calls this (it holds the barriers).
// rho0 (optional): the window starts from feq(rho0), formed on load exactly
// as the init kernel stores it, instead of from src.  rho_out (optional): the
// density of every stored site is written too, as the readout computes it.
// Both 16-byte aligned.
template <int Q, int P, int B>
__device__ __forceinline__ void window_lane(const char* __restrict__ src, char* __restrict__ dst, int64_t n,
                                            int64_t p, int64_t j0, int64_t kl0, int64_t k_lo, int64_t valid,
                                            int s, double* xch, const Coef& cf,
                                            const double* __restrict__ rho0 = nullptr,
                                            double* __restrict__ rho_out = nullptr)
{
    using E = Engine<Q, P, B, kTileLD>;
    using PL = typename E::PL;
    constexpr int L = kTileLD;
    const int lane = threadIdx.x;
    typename E::Site x[B];
    // the vector accesses (16 bytes on double rows, 8 on float rows) need an
    // even first site (rows are 256-byte aligned and their pitch is a
    // multiple of 64 sites).  With one 4-byte access per site, the write-back
    // of float rows (lanes 40 bytes apart) reached memory as several times
    // its bytes.
    const bool inside = j0 >= 0 && j0 + B <= n;
    const bool even = (j0 & 1) == 0;
    if (rho0) {
        if (inside && even) {
            const d2v* r = reinterpret_cast<const d2v*>(rho0 + j0);
            unroll<B / 2>([&](auto K) {
                const d2v v = r[K];
                x[2 * K] = PL::equilibrium(v.x, cf);
                x[2 * K + 1] = PL::equilibrium(v.y, cf);
            });
        } else {
            unroll<B>([&](auto Bi) { x[Bi] = PL::equilibrium(rho0[wrap_site(j0 + Bi, n)], cf); });
        }
    } else if (inside && even) {
        E::PL::template load_vec<B>(src, p, j0, x);
    } else if (inside) {
        unroll<B>([&](auto Bi) { x[Bi] = E::PL::load(src, p, j0 + Bi); });
    } else {
        unroll<B>([&](auto Bi) { x[Bi] = E::PL::load(src, p, wrap_site(j0 + Bi, n)); });
    }
    const int left = lane == 0 ? L - 1 : lane - 1;
    const int right = lane + 1 == L ? 0 : lane + 1;
    E::run(x, s, xch, lane, left, right, true, cf);
    if (kl0 >= k_lo && kl0 + B <= k_lo + valid && inside && even) {
        E::PL::template store_vec<B>(dst, p, j0, x);
    } else {
        unroll<B>([&](auto Bi) {
            const int64_t k = kl0 + Bi;
            const int64_t j = j0 + Bi;      // >= 0 for every stored slot
            if (k >= k_lo && k < k_lo + valid && j < n) E::PL::store(dst, p, j, x[Bi]);
        });
    }
    if (rho_out) {
        if (kl0 >= k_lo && kl0 + B <= k_lo + valid && inside && even) {
            d2v* r = reinterpret_cast<d2v*>(rho_out + j0);
            unroll<B / 2>([&](auto K) {
                d2v v;
                v.x = PL::density(x[2 * K]);
                v.y = PL::density(x[2 * K + 1]);
                r[K] = v;
            });
        } else {
            unroll<B>([&](auto Bi) {
                const int64_t k = kl0 + Bi;
                const int64_t j = j0 + Bi;
                if (k >= k_lo && k < k_lo + valid && j < n) rho_out[j] = PL::density(x[Bi]);
            });
        }
    }
}

// Large periodic lattice: tile t writes sites [t T, t T + T) from a window of
// B * 256 sites starting H s sites earlier.
// rho0 / rho_out (may be null): the first and the last launch of a solve
// start from feq(rho0) and also write the density (see window_lane).
template <int Q, int P, int B>
__global__ __launch_bounds__(kTileLD) void k_tile(const char* __restrict__ src, char* __restrict__ dst,
                                                  int64_t n, int64_t p, int s, int64_t T, Coef cf,
                                                  const double* __restrict__ rho0, double* __restrict__ rho_out)
{
    extern __shared__ double xch[];
    constexpr int H = halo_of(Q);
    const int64_t ws = xcd_block(blockIdx.x, gridDim.x) * T - (int64_t)H * s;
    const int64_t kl0 = (int64_t)threadIdx.x * B;
    window_lane<Q, P, B>(src, dst, n, p, ws + kl0, kl0, (int64_t)H * s, T, s, xch, cf, rho0, rho_out);
}

// Waves per SIMD the ensemble kernel is compiled for: three (the LDS
// exchange areas of three workgroups fit a CU) where that costs at most a few
// spills outside the step loop; two for 12 FP64 sites per lane (228
// registers); split storage needs too many registers.
constexpr int ens_waves_per_simd(int p, int b) { return p == kSPLIT ? 1 : (b == 12 ? 2 : 3); }

// Ensemble: workgroup w runs window hdr[w], whose segments seg[first ..
// first + nseg) occupy consecutive lane ranges; each segment is one tile of
// one instance with its own halo, so several small instances share a window.
// Lanes past the last segment's tile carry junk that is never stored.  The
// window's coefficient set is uniform over the workgroup (scalar loads).
template <int Q, int P, int B>
__global__ __launch_bounds__(kTileLD) __attribute__((amdgpu_waves_per_eu(ens_waves_per_simd(P, B)))) void k_ens(const WinHdr* __restrict__ hdr,
                                                 const SegDesc* __restrict__ seg, const Coef* __restrict__ coefs)
{
    extern __shared__ double xch[];
    constexpr int H = halo_of(Q);
    const WinHdr h = hdr[blockIdx.x];
    const Coef cf = coefs[h.coef];
    const int lane = threadIdx.x;
    int my = 0;
    for (int k = 1; k < h.nseg; k++)
        if (seg[h.first_seg + k].lane_lo <= lane) my = k;
    const SegDesc d = seg[h.first_seg + my];
    const int64_t kl0 = (int64_t)(lane - d.lane_lo) * B;
    window_lane<Q, P, B>(reinterpret_cast<const char*>(d.src), reinterpret_cast<char*>(d.dst), d.n, d.pitch,
                         d.start + kl0, kl0,
                         (int64_t)H * h.steps, d.valid, h.steps, xch, cf);
}

// ---------------------------------------------------------------- one lattice over many workgroups

constexpr int kSpanLD = 64;      // one wave per workgroup: lanes trade values by DPP, no barrier
// Sites per lane of a SPAN window: few, so that a step's dependency chain is
// short; a narrower window exchanges more often, which measures as the better
// trade for the lattices SPAN serves.  Two for the population states of both
// schemes (a D1Q7 population with |c| = 3 then moves up to two lanes per
// step); max|c| for the rho-only state, whose exchange sends densities to the
// neighbouring lanes only.
__host__ __device__ constexpr int span_b_of(int q, int p) { return p == kRHO ? halo_of(q) : 2; }
constexpr int kSpinLimit = 1 << 21;
// Wait before the first poll of an exchange, in units of 64 clocks: about as
// long as the neighbours' stores take to become visible, which grows with
// the words an owner publishes (two sites of 7 or 5 populations per lane).
// Shorter waits spend memory traffic on polls that find sentinels, longer
// ones idle (D1Q7 N = 4096, 16 steps between exchanges: 4 / 6 / 8 / 12 / 16
// units ran 18.2 / 18.8 / 19.5 / 19.1 / 18.5 GLUPS).
__host__ __device__ constexpr int first_poll_delay(int q) { return q == 7 ? 8 : 6; }

// Control words of the multi-workgroup kernel (device memory, kept by the
// lattice across launches): the abort word of the current launch, a sticky
// error word (set with it, cleared only when the state is replaced), a word
// the first owner to raise the abort of a launch claims, and the number of
// launches that stopped early since the lattice was created (never cleared).
constexpr int kCtlAbort = 0, kCtlSticky = 1, kCtlRaised = 2, kCtlAborts = 3, kCtlWords = 64;

// Edge slots.  At exchange c owner w stores its own sites, once, into slot
// (c, w); its left neighbour reads the first H s of them, its right
// neighbour the last H s.  Within one launch every slot word is written once;
// before the launch the whole area holds a sentinel no arithmetic produces (a
// signalling NaN with a fixed payload).  Writer and readers use relaxed
// device-scope atomic accesses per word, so a reader needs no flag and no
// fence: a word that no longer holds the sentinel holds its one value of this
// launch.
// s_waitcnt vmcnt(0) with expcnt and lgkmcnt left at their maximum (gfx9
// encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVmcnt0 = 0x0F70;

constexpr unsigned long long kSent64 = 0x7FF4A5A5A5A5A5A5ull;
constexpr unsigned int kSent32 = 0x7FA5A5A5u;

__device__ __forceinline__ void st_sync(double* a, double v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(a), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sync(float* a, float v)
{
    __hip_atomic_store(reinterpret_cast<unsigned int*>(a), __float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool ld_sync(const double* a, double& v)
{
    const unsigned long long u = __hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<double*>(a)),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v = __longlong_as_double((long long)u);
    return u != kSent64;
}
__device__ __forceinline__ bool ld_sync(const float* a, float& v)
{
    const unsigned int u = __hip_atomic_load(reinterpret_cast<unsigned int*>(const_cast<float*>(a)),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v = __uint_as_float(u);
    return u != kSent32;
}
__device__ __forceinline__ void st_sent(double* a)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(a), kSent64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sent(float* a)
{
    __hip_atomic_store(reinterpret_cast<unsigned int*>(a), kSent32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Word-wise access to one site of a state-format copy (pitch p): every word
// of the site through fn(pointer, member).
template <int Q, int P>
struct SiteWords;

template <int Q>
struct SiteWords<Q, kFP64> {
    template <class S, class F>
    __device__ static __forceinline__ void each(char* st, int64_t p, int64_t j, S& x, F&& fn)
    {
        unroll<Q>([&](auto I) { fn(reinterpret_cast<double*>(st) + I * p + j, x.s[I]); });
    }
};
template <int Q>
struct SiteWords<Q, kFP32> {
    template <class S, class F>
    __device__ static __forceinline__ void each(char* st, int64_t p, int64_t j, S& x, F&& fn)
    {
        unroll<Q>([&](auto I) { fn(reinterpret_cast<float*>(st) + I * p + j, x.s[I]); });
    }
};
template <int Q>
struct SiteWords<Q, kSPLIT> {
    template <class S, class F>
    __device__ static __forceinline__ void each(char* st, int64_t p, int64_t j, S& x, F&& fn)
    {
        fn(reinterpret_cast<double*>(st) + j, x.rho);
        float* nb = reinterpret_cast<float*>(st + p * (int64_t)sizeof(double));
        unroll<Q>([&](auto I) { fn(nb + I * p + j, x.n[I]); });
    }
};
template <int Q>
struct SiteWords<Q, kRHO> {
    template <class S, class F>
    __device__ static __forceinline__ void each(char* st, int64_t, int64_t j, S& x, F&& fn)
    {
        fn(reinterpret_cast<double*>(st) + j, x.rho);
    }
};

template <int Q, int P>
__device__ __forceinline__ void site_store_sync(char* st, int64_t p, int64_t j, const typename Pol<Q, P>::Site& x)
{
    typename Pol<Q, P>::Site y = x;
    SiteWords<Q, P>::each(st, p, j, y, [](auto* a, auto v) { st_sync(a, v); });
}

// true when no word of the site holds the sentinel (all loads are issued
// before any result is tested)
template <int Q, int P>
__device__ __forceinline__ bool site_load_sync(char* st, int64_t p, int64_t j, typename Pol<Q, P>::Site& x)
{
    int missing = 0;
    SiteWords<Q, P>::each(st, p, j, x, [&](auto* a, auto& v) { missing |= ld_sync(a, v) ? 0 : 1; });
    return missing == 0;
}

template <int Q, int P>
__device__ __forceinline__ void site_store_sentinel(char* st, int64_t p, int64_t j)
{
    typename Pol<Q, P>::Site y{};
    SiteWords<Q, P>::each(st, p, j, y, [](auto* a, auto) { st_sent(a); });
}

// Layout of an edge slot: the own sites of the writer (window slots
// [hs, hs + mmax)) occupy lanes first .. first + lanes - 1; slot k = lane B + b
// sits at b * lanes + (lane - first) of each row, so each store and poll
// instruction covers consecutive words.  Rows hold `pitch` words.
struct SpanSlot {
    int64_t first, lanes, b, pitch;
    __host__ __device__ int64_t pos(int64_t k) const { return (k % b) * lanes + (k / b - first); }
};
__host__ __device__ inline SpanSlot span_slot_shape(int b, int64_t hs, int64_t mmax)
{
    SpanSlot s;
    s.b = b;
    s.first = hs / b;
    s.lanes = (hs + mmax - 1) / b - s.first + 1;
    s.pitch = (b * s.lanes + 15) / 16 * 16;
    return s;
}

__device__ __forceinline__ void span_raise_abort(int* ctl, int lane)
{
    if (lane == 0) {
        int expect = 0;
        if (__hip_atomic_compare_exchange_strong(ctl + kCtlRaised, &expect, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            __hip_atomic_fetch_add(ctl + kCtlAborts, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(ctl + kCtlSticky, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(ctl + kCtlAbort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// First site of owner w when n sites are split over nwg owners, and the owner
// of site j (0 <= j < n): the largest w with o(w) <= j.
__device__ __forceinline__ int64_t span_first(int64_t n, int nwg, int64_t w) { return n * w / nwg; }
__device__ __forceinline__ int span_owner(int64_t n, int nwg, int64_t j)
{
    int64_t w = j * nwg / n;
    while (w + 1 < nwg && span_first(n, nwg, w + 1) <= j) w++;
    while (w > 0 && span_first(n, nwg, w) > j) w--;
    return (int)w;
}

// Workgroup w owns sites [o_w, o_w + M_w) of the lattice and holds them, plus
// H s halo sites on each side, in its registers (window slot k <-> site
// o_w - H s + k); a halo may span several owners.  The state is read from src
// at the start of a launch and written to dst at its end.  Every s steps each
// owner stores its own sites to its edge slot of this exchange and loads its
// halo from the slots of the owners of those sites, polling until no word
// holds the sentinel.  Every wait is bounded; on timeout a workgroup raises
// the abort word and every workgroup stops.
template <int Q, int P, bool FIX>
__global__ __launch_bounds__(kSpanLD) void k_span(const char* __restrict__ src, char* __restrict__ dst, int64_t n,
                                                  int64_t p, int nwg, int64_t steps, int s, char* __restrict__ ebase,
                                                  int64_t ecopy, int64_t epitch, int64_t slots,
                                                  int* __restrict__ ctl, Coef cf, double rho_l, double rho_r)
{
    using E = Engine<Q, P, span_b_of(Q, P), kSpanLD>;
    using PL = typename E::PL;
    using Site = typename E::Site;
    constexpr int B = span_b_of(Q, P);
    double* xch = nullptr;   // single wave: the engine exchanges by DPP
    // consecutive owners share an XCD (workgroups are dealt round-robin to 8 XCDs)
    const int per = (nwg + 7) / 8;
    const int w = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (w >= nwg) return;
    // a lattice whose earlier launch stopped early holds no valid state
    // until it is replaced: leave it (and its error) as it is
    if (__hip_atomic_load(ctl + kCtlSticky, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t o = span_first(n, nwg, w);
    const int64_t M = span_first(n, nwg, w + 1) - o;
    const int hs = E::H * s;
    const int lane = threadIdx.x;
    const int left = lane == 0 ? kSpanLD - 1 : lane - 1;
    const int right = lane + 1 == kSpanLD ? 0 : lane + 1;
    auto slot = [&](int64_t chunk, int who) { return ebase + (chunk * nwg + who) * ecopy; };
    const SpanSlot sl = span_slot_shape(B, hs, (n + nwg - 1) / nwg);
    auto pos = [&](int64_t k) { return sl.pos(k); };

    // where each halo slot of this lane comes from: the owner of its site and
    // that owner's window slot of it (slots outside the halo read the first
    // word of this owner's own slot and ignore it)
    int src_w[B];
    int64_t idx[B];
    bool want[B];
    unroll<B>([&](auto Bi) {
        const int64_t k = (int64_t)lane * B + Bi;
        want[Bi] = k < hs || k >= hs + M;
        src_w[Bi] = w;
        idx[Bi] = 0;
        if (want[Bi]) {
            const int64_t j = wrap_site(o - hs + k, n);
            const int ow = span_owner(n, nwg, j);
            src_w[Bi] = ow;
            idx[Bi] = pos(hs + (j - span_first(n, nwg, ow)));
        }
    });

    Site x[B];
    unroll<B>([&](auto Bi) {
        const int64_t k = (int64_t)lane * B + Bi;
        x[Bi] = PL::load(src, p, wrap_site(o - hs + k, n));
    });
    // fixed ends: sites <= 0 and >= n-1 (boundary sites and the ghosts
    // beyond them) hold the end-value equilibria after every step; only the
    // owners whose window reaches an end apply it
    const int64_t j0 = o - hs + (int64_t)lane * B;
    const bool touches = FIX && (o - hs <= 0 || o + M + hs >= n - 1);
    const Site eq_l = PL::equilibrium(rho_l, cf), eq_r = PL::equilibrium(rho_r, cf);
    auto fix = [&](Site (&y)[B]) {
        if (touches) {
            unroll<B>([&](auto Bi) {
                const int64_t j = j0 + Bi;
                if (j <= 0) y[Bi] = eq_l;
                else if (j >= n - 1) y[Bi] = eq_r;
            });
        }
    };
    if constexpr (FIX) fix(x);
    int64_t done = 0;
    for (int64_t c = 0; done < steps; c++) {
        const int sc = (int)(steps - done < s ? steps - done : s);
        if constexpr (FIX) E::run(x, sc, xch, lane, left, right, true, cf, fix);
        else E::run(x, sc, xch, lane, left, right, true, cf);
        done += sc;
        if (done >= steps) break;
        if (c >= slots) {   // the host sizes launches to their slots; stop rather than overrun
            span_raise_abort(ctl, lane);
            return;
        }
        // Publish own sites (one store per word).  No memory access of this
        // wave is outstanding here (the halo loads were consumed by the last
        // chunk); saying so keeps the compiler from waiting for them between
        // these stores, which the counter it waits on also counts.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        unroll<B>([&](auto Bi) {
            const int64_t k = (int64_t)lane * B + Bi;
            if (k >= hs && k < hs + M) site_store_sync<Q, P>(slot(c, w), epitch, pos(k), x[Bi]);
        });
        // Receive the halo: every lane loads (so all loads of a poll are in
        // flight together: one memory round trip per poll), polling until no
        // wanted word holds the sentinel.  The neighbours' stores leave at the
        // same time as ours, so a first poll issued at once mostly reaches
        // memory before them: wait a little first.
        __builtin_amdgcn_s_sleep(first_poll_delay(Q));
        for (int spin = 0;; spin++) {
            Site y[B];
            bool got[B];
            unroll<B>([&](auto Bi) { got[Bi] = site_load_sync<Q, P>(slot(c, src_w[Bi]), epitch, idx[Bi], y[Bi]); });
            const int ab = __hip_atomic_load(ctl + kCtlAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bool ready = true;
            unroll<B>([&](auto Bi) { ready = ready && (got[Bi] || !want[Bi]); });
            const bool all_ready = __builtin_amdgcn_ballot_w64(!ready) == 0;
            // an abort raised anywhere stops every owner at its next poll
            if (__builtin_amdgcn_readfirstlane(ab) || (!all_ready && spin >= kSpinLimit)) {
                span_raise_abort(ctl, lane);
                return;
            }
            if (all_ready) {
                unroll<B>([&](auto Bi) {
                    if (want[Bi]) x[Bi] = y[Bi];
                });
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if constexpr (FIX) fix(x);
    }
    unroll<B>([&](auto Bi) {
        const int64_t k = (int64_t)lane * B + Bi;
        if (k >= hs && k < hs + M) PL::store(dst, p, o + k - hs, x[Bi]);
    });
}

// Before each launch: clear the abort word and its claim.
__global__ void k_span_prep(int* ctl)
{
    if (threadIdx.x == 0) {
        ctl[kCtlAbort] = 0;
        ctl[kCtlRaised] = 0;
    }
}

// Sentinel in the words of `copies` edge copies that hold own sites: window
// slots [hs, hs + sites) at their slot positions.
template <int Q, int P>
__global__ __launch_bounds__(256) void k_span_fill(char* ebase, int64_t ecopy, int64_t epitch, int64_t copies,
                                                   int hs, int sites)
{
    const SpanSlot sl = span_slot_shape(span_b_of(Q, P), hs, sites);
    const int64_t total = copies * sites;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t c = i / sites, k = hs + (i - c * sites);
        site_store_sentinel<Q, P>(ebase + c * ecopy, epitch, sl.pos(k));
    }
}

__global__ void k_span_set_ctl(int* ctl, int index, int value)
{
    if (threadIdx.x == 0) ctl[index] = value;
}

__global__ void k_span_init_ctl(int* ctl, int count)
{
    for (int i = threadIdx.x; i < count; i += blockDim.x) ctl[i] = 0;
}

// ---------------------------------------------------------------- trajectory pairs

// Benettin renormalisation of FP64 trajectory pairs (one workgroup per pair):
// d = || S_pert - S_ref ||_2 over the Q x n post-collision populations, summed
// in a fixed order (strided per thread, then a tree over the workgroup);
// S_pert <- S_ref + (S_pert - S_ref) delta / d; log_accum[slot] += ln(d / delta).
// A zero or non-finite d leaves the pair unchanged and stores NaN.
constexpr int kPairLD = 1024;

template <int Q>
__global__ __launch_bounds__(kPairLD) void k_pair_renorm(const PairDesc* __restrict__ pd,
                                                        double delta, double* __restrict__ log_accum)
{
    __shared__ double red[kPairLD];
    __shared__ double scale_sh;
    const PairDesc d = pd[blockIdx.x];
    const double* r = reinterpret_cast<const double*>(d.ref);
    double* x = reinterpret_cast<double*>(d.pert);
    const int t = threadIdx.x;
    const int64_t total = (int64_t)Q * d.n;
    double ss = 0.0;
    for (int64_t e = t; e < total; e += kPairLD) {
        const int64_t i = e / d.n, j = e - i * d.n;
        const double diff = x[i * d.pitch + j] - r[i * d.pitch + j];
        ss = __builtin_fma(diff, diff, ss);
    }
    red[t] = ss;
    __syncthreads();
    for (int h = kPairLD / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) {
        const double dist = sqrt(red[0]);
        const bool ok = dist > 0.0 && __builtin_isfinite(dist);
        scale_sh = ok ? delta / dist : 0.0;
        log_accum[d.slot] = ok ? log_accum[d.slot] + log(dist / delta) : __builtin_nan("");
    }
    __syncthreads();
    const double sc = scale_sh;
    if (sc == 0.0) return;
    for (int64_t e = t; e < total; e += kPairLD) {
        const int64_t i = e / d.n, j = e - i * d.n;
        const double ref = r[i * d.pitch + j];
        x[i * d.pitch + j] = __builtin_fma(x[i * d.pitch + j] - ref, sc, ref);
    }
}

int launch_pair_renorm(int q, const PairDesc* desc, int npairs, double delta, double* log_accum, void* stream)
{
    if (npairs <= 0) return 0;
    if (q == 5) k_pair_renorm<5><<<npairs, kPairLD, 0, (hipStream_t)stream>>>(desc, delta, log_accum);
    else k_pair_renorm<7><<<npairs, kPairLD, 0, (hipStream_t)stream>>>(desc, delta, log_accum);
    return (int)hipGetLastError();
}

// Lyapunov spectrum: renormalisation of a reference trajectory and K
// perturbed copies (one workgroup per group).  With v_m = S_pert[m] - S_ref
// over the Q x n post-collision populations, the Gram matrix G_ab = v_a . v_b
// (fixed-order sums: strided per thread, then a tree over the workgroup) is
// factored G = R^T R (Cholesky, R upper triangular with positive diagonal),
// so V = U R with orthonormal U; then S_pert[m] <- S_ref + delta u_m and
// log_accum[slot + m] += ln(R_mm / delta).  If R is not positive definite and
// finite the group is left unchanged and NaN is stored.
template <int Q, int K>
__global__ __launch_bounds__(kPairLD) void k_group_orth(const GroupDesc* __restrict__ gd,
                                                       const uint64_t* __restrict__ pert, double delta,
                                                       double* __restrict__ log_accum)
{
    constexpr int NP = K * (K + 1) / 2;
    __shared__ double red[kPairLD];
    __shared__ double gram[NP];
    __shared__ double rm[K][K];
    __shared__ int ok_sh;
    const GroupDesc g = gd[blockIdx.x];
    const double* r = reinterpret_cast<const double*>(g.ref);
    double* x[K];
    unroll<K>([&](auto M) { x[M] = reinterpret_cast<double*>(pert[g.first + M]); });
    const int t = threadIdx.x;
    const int64_t total = (int64_t)Q * g.n;
    double acc[NP];
    unroll<NP>([&](auto P) { acc[P] = 0.0; });
    for (int64_t e = t; e < total; e += kPairLD) {
        const int64_t i = e / g.n, idx = i * g.pitch + (e - i * g.n);
        const double rv = r[idx];
        double v[K];
        unroll<K>([&](auto M) { v[M] = x[M][idx] - rv; });
        unroll<K>([&](auto A) {
            unroll<K>([&](auto B) {
                constexpr int a = A, b = B;
                if constexpr (b >= a) {
                    constexpr int P = a * K - a * (a - 1) / 2 + (b - a);   // packed upper triangle
                    acc[P] = __builtin_fma(v[a], v[b], acc[P]);
                }
            });
        });
    }
    unroll<NP>([&](auto P) {
        red[t] = acc[P];
        __syncthreads();
        for (int h = kPairLD / 2; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        if (t == 0) gram[P] = red[0];
        __syncthreads();
    });
    if (t == 0) {
        // packed index of (a, b), a <= b, in the row-major upper triangle
        auto at = [](int a, int b) { return a * K - a * (a - 1) / 2 + (b - a); };
        bool ok = true;
        for (int m = 0; m < K && ok; m++) {
            double d = gram[at(m, m)];
            for (int l = 0; l < m; l++) d -= rm[l][m] * rm[l][m];
            const double rmm = d > 0.0 ? sqrt(d) : 0.0;
            ok = rmm > 0.0 && __builtin_isfinite(rmm);
            rm[m][m] = rmm;
            for (int c = m + 1; c < K && ok; c++) {
                double o = gram[at(m, c)];
                for (int l = 0; l < m; l++) o -= rm[l][m] * rm[l][c];
                rm[m][c] = o / rmm;
            }
        }
        for (int m = 0; m < K; m++)
            log_accum[g.slot + m] = ok ? log_accum[g.slot + m] + log(rm[m][m] / delta) : __builtin_nan("");
        ok_sh = ok ? 1 : 0;
    }
    __syncthreads();
    if (!ok_sh) return;
    double rr[K][K];
    unroll<K>([&](auto A) { unroll<K>([&](auto B) { rr[A][B] = (B >= A) ? rm[A][B] : 0.0; }); });
    for (int64_t e = t; e < total; e += kPairLD) {
        const int64_t i = e / g.n, idx = i * g.pitch + (e - i * g.n);
        const double rv = r[idx];
        double u[K];
        unroll<K>([&](auto M) {
            double v = x[M][idx] - rv;
            unroll<K>([&](auto L) { if constexpr (L < M) v -= u[L] * rr[L][M]; });
            u[M] = v / rr[M][M];
        });
        unroll<K>([&](auto M) { x[M][idx] = __builtin_fma(delta, u[M], rv); });
    }
}

template <int Q>
static int group_orth_q(int k, const GroupDesc* desc, const uint64_t* pert, int ngroups, double delta,
                        double* log_accum, hipStream_t st)
{
    switch (k) {
    case 1: k_group_orth<Q, 1><<<ngroups, kPairLD, 0, st>>>(desc, pert, delta, log_accum); break;
    case 2: k_group_orth<Q, 2><<<ngroups, kPairLD, 0, st>>>(desc, pert, delta, log_accum); break;
    case 3: k_group_orth<Q, 3><<<ngroups, kPairLD, 0, st>>>(desc, pert, delta, log_accum); break;
    case 4: k_group_orth<Q, 4><<<ngroups, kPairLD, 0, st>>>(desc, pert, delta, log_accum); break;
    case 5: k_group_orth<Q, 5><<<ngroups, kPairLD, 0, st>>>(desc, pert, delta, log_accum); break;
    case 6: k_group_orth<Q, 6><<<ngroups, kPairLD, 0, st>>>(desc, pert, delta, log_accum); break;
    case 7: k_group_orth<Q, 7><<<ngroups, kPairLD, 0, st>>>(desc, pert, delta, log_accum); break;
    case 8: k_group_orth<Q, 8><<<ngroups, kPairLD, 0, st>>>(desc, pert, delta, log_accum); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_group_orth(int q, int k, const GroupDesc* desc, const uint64_t* pert, int ngroups, double delta,
                      double* log_accum, void* stream)
{
    if (ngroups <= 0) return 0;
    if (q == 5) return group_orth_q<5>(k, desc, pert, ngroups, delta, log_accum, (hipStream_t)stream);
    return group_orth_q<7>(k, desc, pert, ngroups, delta, log_accum, (hipStream_t)stream);
}

// ---------------------------------------------------------------- readout and diagnostics

// err (may be null): the lattice's sticky error word; while it is set the
// state is not valid and the readout is NaN.
template <int Q, int P>
__global__ __launch_bounds__(256) void k_read_rho(const char* __restrict__ st, int64_t n, int64_t p,
                                                  double* __restrict__ out, const int* __restrict__ err)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    out[j] = (err && *err) ? __builtin_nan("") : PL::density(PL::load(st, p, j));
}

// Density readout of many lattices in one launch (block row y: instance d[y]).
template <int Q, int P>
__global__ __launch_bounds__(256) void k_read_many(const InstDesc* __restrict__ d,
                                                   double* __restrict__ rho)
{
    using PL = Pol<Q, P>;
    const InstDesc e = d[blockIdx.y];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < e.n) rho[e.rho_off + j] = PL::density(PL::load(reinterpret_cast<const char*>(e.state), e.pitch, j));
}

// out is dense Q x n
template <int Q, int P>
__global__ __launch_bounds__(256) void k_read_f(const char* __restrict__ st, int64_t n, int64_t p,
                                                double* __restrict__ out, int pre, Coef cf,
                                                const int* __restrict__ err)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const bool bad = err && *err;
    unroll<Q>([&](auto I) {
        const int64_t s = pre ? wrap_site(j - vel(I), n) : j;
        out[I * n + j] = bad ? __builtin_nan("") : PL::template pop_g<I>(st, p, s, cf);
    });
}

template <int Q, int P>
__global__ __launch_bounds__(256) void k_write_f(char* st, int64_t n, int64_t p, const double* __restrict__ in,
                                                 Coef cf)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double f[Q];
    unroll<Q>([&](auto I) { f[I] = in[I * n + j]; });
    PL::store(st, p, j, PL::from_f(f, cf));
}

__global__ void k_zero_int(int* p) { *p = 0; }

constexpr int kDiagBlocks = 256;

// Stage 1: block b sums the densities of sites b*256 + t + k*65536 (fixed
// order), then a fixed tree over its 256 threads.
template <int Q, int P>
__global__ __launch_bounds__(256) void k_diag1(const char* __restrict__ st, int64_t n, int64_t p, double* partial,
                                               int* flag)
{
    using PL = Pol<Q, P>;
    __shared__ double red[256];
    double acc = 0.0;
    bool ok = true;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)kDiagBlocks * 256) {
        const auto x = PL::load(st, p, j);
        acc += PL::density(x);
        ok = ok && PL::finite(x);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (unsigned w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
    if (!ok) atomicOr(flag, 1);
}

__global__ void k_diag2(const double* partial, double* out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < kDiagBlocks; b++) s += partial[b];
        *out = s;
    }
}

// ---------------------------------------------------------------- host launchers

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

#define KSLB_DISPATCH_QP(q, prec, CALL)                                  \
    do {                                                                 \
        if ((q) == 5) {                                                  \
            if ((prec) == kFP64) { constexpr int Q_ = 5, P_ = kFP64; CALL; } \
            else if ((prec) == kFP32) { constexpr int Q_ = 5, P_ = kFP32; CALL; } \
            else if ((prec) == kSPLIT) { constexpr int Q_ = 5, P_ = kSPLIT; CALL; } \
            else { constexpr int Q_ = 5, P_ = kRHO; CALL; }               \
        } else {                                                         \
            if ((prec) == kFP64) { constexpr int Q_ = 7, P_ = kFP64; CALL; } \
            else if ((prec) == kFP32) { constexpr int Q_ = 7, P_ = kFP32; CALL; } \
            else if ((prec) == kSPLIT) { constexpr int Q_ = 7, P_ = kSPLIT; CALL; } \
            else { constexpr int Q_ = 7, P_ = kRHO; CALL; }               \
        }                                                                \
    } while (0)

int64_t state_pitch(int64_t n) { return (n + 63) / 64 * 64; }

size_t state_copy_bytes(int64_t n, int q, int prec)
{
    const size_t p = (size_t)state_pitch(n);
    size_t b;
    if (prec == kFP64) b = (size_t)q * p * 8;
    else if (prec == kFP32) b = (size_t)q * p * 4;
    else if (prec == kSPLIT) b = p * 8 + (size_t)q * p * 4;
    else b = p * 8;
    return (b + 255) & ~(size_t)255;
}

// Host-side caches below are shared by every lattice and ensemble of the
// process, so each is guarded by its own mutex.  They are fixed-size tables
// (no heap allocation after load), indexed by device ordinal.
constexpr int kMaxDevices = 64;

int max_lds_bytes()
{
    static std::mutex mu;
    static int cached[kMaxDevices] = {};   // 0: not queried yet
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 65536;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] > 0) return cached[dev];
    int v = 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    cached[dev] = v;
    return v;
}

int ring_max_lanes() { return kRingLD; }
int tile_lanes() { return kTileLD; }
int ring_lds_bytes(int q) { return 2 * nx_of(q) * kRingLD * (int)sizeof(double); }
int tile_lds_bytes(int q) { return 2 * nx_of(q) * kTileLD * (int)sizeof(double); }
// (the rho-only engine exchanges fewer values and uses a prefix of these areas)

// Raise a kernel's dynamic LDS limit above 64 KiB, once per device, kernel
// and size (the attribute is per function; the table is process-wide, so it
// is updated under a mutex and lattices on several threads may launch).
static int prep_lds_fn(const void* fn, int bytes)
{
    struct Done {
        int dev;
        const void* fn;
        int bytes;
    };
    static std::mutex mu;
    static Done done[512];   // (device, kernel) -> bytes set; a full table only repeats the call
    static int used = 0;
    if (bytes <= 65536) return 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    std::lock_guard<std::mutex> lock(mu);
    Done* d = nullptr;
    for (int i = 0; i < used; i++)
        if (done[i].dev == dev && done[i].fn == fn) d = &done[i];
    if (d && d->bytes >= bytes) return 0;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return (int)e;
    if (!d && used < 512) d = &done[used++];
    if (d) *d = Done{dev, fn, bytes};
    return 0;
}

template <class K>
static int prep_lds(K kernel, int bytes)
{
    return prep_lds_fn(reinterpret_cast<const void*>(kernel), bytes);
}

int launch_init(int q, int prec, void* state, int64_t n, const double* rho0, const Coef& cf, void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_init<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (char*)state, n, state_pitch(n), rho0, cf)));
    return (int)hipGetLastError();
}

int launch_read_many(int q, int prec, const InstDesc* desc, int count, int64_t max_n, double* rho, void* stream)
{
    constexpr int kMaxRows = 65535;   // grid y limit
    for (int y0 = 0; y0 < count; y0 += kMaxRows) {
        const dim3 grid(blocks_for(max_n), (unsigned)std::min(kMaxRows, count - y0));
        KSLB_DISPATCH_QP(q, prec, (k_read_many<Q_, P_><<<grid, 256, 0, (hipStream_t)stream>>>(desc + y0, rho)));
        int e = (int)hipGetLastError();
        if (e) return e;
    }
    return 0;
}

int launch_init_many(int q, int prec, const InstDesc* desc, int count, int64_t max_n, const Coef* coefs,
                     const double* rho, void* stream)
{
    constexpr int kMaxRows = 65535;   // grid y limit
    for (int y0 = 0; y0 < count; y0 += kMaxRows) {
        const dim3 grid(blocks_for(max_n), (unsigned)std::min(kMaxRows, count - y0));
        KSLB_DISPATCH_QP(q, prec, (k_init_many<Q_, P_><<<grid, 256, 0, (hipStream_t)stream>>>(desc + y0, coefs, rho)));
        int e = (int)hipGetLastError();
        if (e) return e;
    }
    return 0;
}

int launch_plain(int q, int prec, const void* src, void* dst, int64_t n, const Coef& cf, void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_plain<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (const char*)src, (char*)dst, n, state_pitch(n), cf)));
    return (int)hipGetLastError();
}

template <int Q, int P, int B>
static int ring_one(const void* src, void* dst, int64_t n, int64_t steps, const Coef& cf, void* stream)
{
    const int L = (int)(n / B);
    const int lanes = ((L + 63) / 64) * 64;
    if (L < 1 || lanes > kRingLD || (int64_t)L * B != n) return (int)hipErrorInvalidValue;
    const int lds = ring_lds_bytes(Q);
    int e = prep_lds(k_ring<Q, P, B>, lds);
    if (e) return e;
    k_ring<Q, P, B><<<1, lanes, lds, (hipStream_t)stream>>>((const char*)src, (char*)dst, (int)n, state_pitch(n),
                                                           steps, cf);
    return (int)hipGetLastError();
}

int launch_ring(int q, int prec, int B, const void* src, void* dst, int64_t n, int64_t steps,
                const Coef& cf, void* stream)
{
    if (B == 4) { KSLB_DISPATCH_QP(q, prec, return (ring_one<Q_, P_, 4>(src, dst, n, steps, cf, stream))); }
    if (B == 8) { KSLB_DISPATCH_QP(q, prec, return (ring_one<Q_, P_, 8>(src, dst, n, steps, cf, stream))); }
    return (int)hipErrorInvalidValue;
}

template <int Q, int P, int B>
static int tile_one(const void* src, void* dst, int64_t n, int s, const Coef& cf, void* stream,
                    const double* rho0, double* rho_out)
{
    const int64_t W = (int64_t)kTileLD * B;
    const int64_t T = W - 2 * (int64_t)halo_of(Q) * s;
    if (T <= 0 || s < 1) return (int)hipErrorInvalidValue;
    const int64_t tiles = (n + T - 1) / T;
    const int lds = tile_lds_bytes(Q);
    int e = prep_lds(k_tile<Q, P, B>, lds);
    if (e) return e;
    k_tile<Q, P, B><<<(unsigned)tiles, kTileLD, lds, (hipStream_t)stream>>>((const char*)src, (char*)dst, n,
                                                                           state_pitch(n), s, T, cf, rho0, rho_out);
    return (int)hipGetLastError();
}

// Sites per lane of the tiled kernel, one width per storage, from sweeps on
// N = 2^24: 12 for FP64 (228 registers for D1Q7, two waves per SIMD: a
// 3072-site window recomputes less halo per stored site than 2048 sites at
// three waves; D1Q7 1060 against 1026 GLUPS, D1Q5 1447 against 1411), 10 for
// FP32 (134 registers, three waves: on two devices 888 and 913 GLUPS against
// 866 and 875 at 8 sites), 32 for the rho-only state (154 registers, three
// waves: 1931 against 1844 GLUPS at 16, D1Q5 2371 against 2309), 8 for split.
__host__ __device__ constexpr int tile_b_of(int p)
{
    return p == kFP64 ? 12 : (p == kFP32 ? 10 : (p == kRHO ? 32 : 8));
}

int tile_sites_per_lane(int prec) { return tile_b_of(prec); }

int launch_tile(int q, int prec, const void* src, void* dst, int64_t n, int s, const Coef& cf, void* stream,
                const double* rho0, double* rho_out)
{
    KSLB_DISPATCH_QP(q, prec, return (tile_one<Q_, P_, tile_b_of(P_)>(src, dst, n, s, cf, stream, rho0, rho_out)));
    return (int)hipErrorInvalidValue;
}

template <int Q, int P, int B>
static int ens_one(const WinHdr* hdr, const SegDesc* seg, int nwin, const Coef* cf, void* stream)
{
    const int lds = tile_lds_bytes(Q);
    int e = prep_lds(k_ens<Q, P, B>, lds);
    if (e) return e;
    k_ens<Q, P, B><<<(unsigned)nwin, kTileLD, lds, (hipStream_t)stream>>>(hdr, seg, cf);
    return (int)hipGetLastError();
}

int launch_ens(int q, int prec, int B, const WinHdr* hdr, const SegDesc* seg, int nwin,
               const Coef* cf, void* stream)
{
    if (nwin <= 0) return 0;
    if (B == 4) { KSLB_DISPATCH_QP(q, prec, return (ens_one<Q_, P_, 4>(hdr, seg, nwin, cf, stream))); }
    if (B == 8) { KSLB_DISPATCH_QP(q, prec, return (ens_one<Q_, P_, 8>(hdr, seg, nwin, cf, stream))); }
    if (B == 12 && prec == kFP64) {
        if (q == 5) return ens_one<5, kFP64, 12>(hdr, seg, nwin, cf, stream);
        return ens_one<7, kFP64, 12>(hdr, seg, nwin, cf, stream);
    }
    if (B == 10 && prec == kFP32) {
        if (q == 5) return ens_one<5, kFP32, 10>(hdr, seg, nwin, cf, stream);
        return ens_one<7, kFP32, 10>(hdr, seg, nwin, cf, stream);
    }
    if (B == 16 && prec == kRHO) {
        if (q == 5) return ens_one<5, kRHO, 16>(hdr, seg, nwin, cf, stream);
        return ens_one<7, kRHO, 16>(hdr, seg, nwin, cf, stream);
    }
    return (int)hipErrorInvalidValue;
}

int span_lanes() { return kSpanLD; }
int span_sites_per_lane(int q, int prec) { return span_b_of(q, prec); }
int span_ctl_ints() { return kCtlWords; }
int64_t span_edge_copy_bytes(int q, int prec, int64_t n, int nwg, int s)
{
    const SpanSlot sl = span_slot_shape(span_b_of(q, prec), (int64_t)halo_of(q) * s, (n + nwg - 1) / nwg);
    return ((int64_t)state_copy_bytes(sl.pitch, q, prec) + 255) / 256 * 256;
}

int launch_span_ctl_init(int* ctl, int count, void* stream)
{
    k_span_init_ctl<<<1, 256, 0, (hipStream_t)stream>>>(ctl, count);
    return (int)hipGetLastError();
}

int launch_span_set_ctl(int* ctl, int index, int value, void* stream)
{
    k_span_set_ctl<<<1, 64, 0, (hipStream_t)stream>>>(ctl, index, value);
    return (int)hipGetLastError();
}

int span_ctl_error_index() { return kCtlSticky; }
int span_ctl_aborts_index() { return kCtlAborts; }

// SPAN owners the current device keeps resident at once: the occupancy of the
// kernel variant (single-wave workgroups, no LDS) times the compute units.
// Every owner polls for its neighbours, so all must run at once.
int64_t span_device_owners(int q, int prec, bool fixed)
{
    static std::mutex mu;
    static int64_t cached[kMaxDevices][2][4][2];   // (device, q, prec, fixed); 0: not queried yet
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices || prec < 0 || prec > 3) return 0;
    std::lock_guard<std::mutex> lock(mu);
    int64_t& slot = cached[dev][q == 7][prec][fixed ? 1 : 0];
    if (slot > 0) return slot;
    int per_cu = 0, cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) {
        if (fixed) {
            KSLB_DISPATCH_QP(q, prec, (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                           &per_cu, reinterpret_cast<const void*>(k_span<Q_, P_, true>), kSpanLD, 0)));
        } else {
            KSLB_DISPATCH_QP(q, prec, (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                           &per_cu, reinterpret_cast<const void*>(k_span<Q_, P_, false>), kSpanLD, 0)));
        }
    }
    const int64_t v = (e == hipSuccess && per_cu > 0 && cus > 0) ? (int64_t)per_cu * cus : 0;
    slot = v;
    return v;
}

int launch_span(int q, int prec, const void* src, void* dst, int64_t n, int nwg, int64_t steps, int s, char* ebase,
                int64_t ecopy, int64_t slots, int* ctl, const Coef& cf, void* stream, const Ends* ends,
                bool inject_abort)
{
    hipStream_t st = (hipStream_t)stream;
    const int h = halo_of(q);
    const int64_t hs = (int64_t)h * s;
    const int64_t W = (int64_t)kSpanLD * span_b_of(q, prec);
    if (nwg < 2 || s < 1 || steps < 1 || slots < 1) return (int)hipErrorInvalidValue;
    // every owner holds at least one site and its window fits
    const int64_t mmin = n / nwg, mmax = (n + nwg - 1) / nwg;
    if (mmin < 1 || mmax + 2 * hs > W) return (int)hipErrorInvalidValue;
    // the exchanges of this launch fit the slots
    if ((steps + s - 1) / s - 1 > slots) return (int)hipErrorInvalidValue;
    const int64_t epitch = span_slot_shape(span_b_of(q, prec), hs, mmax).pitch;
    if (ecopy < (int64_t)state_copy_bytes(epitch, q, prec)) return (int)hipErrorInvalidValue;
    const int64_t copies = std::min<int64_t>(slots, (steps + s - 1) / s - 1) * nwg;
    k_span_prep<<<1, 64, 0, st>>>(ctl);
    if (inject_abort) k_span_set_ctl<<<1, 64, 0, st>>>(ctl, kCtlAbort, 1);   // failure-path testing
    if (copies > 0) {
        const unsigned fill_blocks = (unsigned)std::min<int64_t>(4096, (copies * mmax + 255) / 256);
        KSLB_DISPATCH_QP(q, prec, (k_span_fill<Q_, P_><<<fill_blocks, 256, 0, st>>>(ebase, ecopy, epitch, copies,
                                                                                   (int)hs, (int)mmax)));
    }
    const int per = (nwg + 7) / 8;
    const unsigned grid = (unsigned)(per * 8);
    if (ends) {
        KSLB_DISPATCH_QP(q, prec, (k_span<Q_, P_, true><<<grid, kSpanLD, 0, st>>>(
                                      (const char*)src, (char*)dst, n, state_pitch(n), nwg, steps, s, ebase, ecopy,
                                      epitch, slots, ctl, cf, ends->rho_l, ends->rho_r)));
    } else {
        KSLB_DISPATCH_QP(q, prec, (k_span<Q_, P_, false><<<grid, kSpanLD, 0, st>>>(
                                      (const char*)src, (char*)dst, n, state_pitch(n), nwg, steps, s, ebase, ecopy,
                                      epitch, slots, ctl, cf, 0.0, 0.0)));
    }
    return (int)hipGetLastError();
}

// Edge slots for callers that cannot allocate (kslb_advance_noalloc): a
// file-scope device array each GPU holds until the process ends.  Host code
// never passes its name to a kernel: in host code the name is a host-side
// stand-in, so the array's device address is looked up once per device and
// that address is what kernels receive.  Every caller on one device shares
// it; calls that overlap on a device race.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

int noalloc_scratch(char** ptr)
{
    static std::mutex mu;
    static char* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        addr[dev] = static_cast<char*>(p);
    }
    *ptr = addr[dev];
    return 0;
}

int launch_plain_fixed(int q, int prec, const void* src, void* dst, int64_t n, const Coef& cf, const Ends& ends,
                       void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_plain_fixed<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (const char*)src, (char*)dst, n, state_pitch(n), cf, ends.rho_l, ends.rho_r)));
    return (int)hipGetLastError();
}

int launch_init_fixed(int q, int prec, void* state, int64_t n, const double* rho0, const Coef& cf, const Ends& ends,
                      void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_init_fixed<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (char*)state, n, state_pitch(n), rho0, cf, ends.rho_l, ends.rho_r)));
    return (int)hipGetLastError();
}

int launch_read_rho(int q, int prec, const void* state, int64_t n, double* out, void* stream, const int* err)
{
    KSLB_DISPATCH_QP(q, prec, (k_read_rho<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (const char*)state, n, state_pitch(n), out, err)));
    return (int)hipGetLastError();
}

int launch_read_f(int q, int prec, const void* state, int64_t n, double* out, int pre, const Coef& cf,
                  void* stream, const int* err)
{
    KSLB_DISPATCH_QP(q, prec, (k_read_f<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (const char*)state, n, state_pitch(n), out, pre, cf, err)));
    return (int)hipGetLastError();
}

int launch_write_f(int q, int prec, void* state, int64_t n, const double* in, const Coef& cf, void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_write_f<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (char*)state, n, state_pitch(n), in, cf)));
    return (int)hipGetLastError();
}

int launch_diag(int q, int prec, const void* state, int64_t n, double* partial, int* flag, double* mass_out,
                void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    k_zero_int<<<1, 1, 0, s>>>(flag);
    KSLB_DISPATCH_QP(q, prec, (k_diag1<Q_, P_><<<kDiagBlocks, 256, 0, s>>>((const char*)state, n,
                                                                          state_pitch(n), partial, flag)));
    k_diag2<<<1, 1, 0, s>>>(partial, mass_out);
    return (int)hipGetLastError();
}

}  // namespace kslb
