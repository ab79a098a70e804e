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
// ping-pong side.  FP64: Q x n doubles.  FP32: Q x n floats.  SPLIT: n
// doubles of rho, then Q x n floats of f_i - feq_i(rho).
//
// Register-resident kernels give each lane B consecutive sites in VGPRs.  A
// step moves data between lanes only at block edges: lane l publishes the
// populations its neighbours pull (the last c sites of each c > 0 population,
// the first |c| of each c < 0 one; 12 doubles for D1Q7, 6 for D1Q5) to a
// double-buffered LDS exchange area, one barrier, then every site is updated
// from registers plus the neighbours' values.
#include <hip/hip_runtime.h>

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

// ---------------------------------------------------------------- precision policies

template <int Q, int P>
struct Pol;

template <int Q>
struct Pol<Q, kFP64> {
    struct Site { double s[Q]; };

    template <int I>
    __device__ static __forceinline__ double pop(const Site& x, const Coef&) { return x.s[I]; }

    template <int I>
    __device__ static __forceinline__ double pop_g(const char* st, int64_t n, int64_t j, const Coef&)
    {
        return reinterpret_cast<const double*>(st)[I * n + j];
    }

    __device__ static __forceinline__ void update(const double (&g)[Q], Site& y, const Coef& cf)
    {
        double rho = g[0];
        unroll<Q - 1>([&](auto I) { rho = rho + g[I + 1]; });
        const double r2 = rho * rho;
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            double eq;
            if constexpr (has_g(i)) eq = __builtin_fma(cf.A[i], rho, cf.B[i] * r2);
            else eq = cf.A[i] * rho;
            y.s[i] = __builtin_fma(cf.a1mw, g[i], eq);
        });
    }

    __device__ static __forceinline__ Site load(const char* st, int64_t n, int64_t j)
    {
        Site x;
        unroll<Q>([&](auto I) { x.s[I] = reinterpret_cast<const double*>(st)[I * n + j]; });
        return x;
    }

    __device__ static __forceinline__ void store(char* st, int64_t n, int64_t j, const Site& x)
    {
        unroll<Q>([&](auto I) { reinterpret_cast<double*>(st)[I * n + j] = x.s[I]; });
    }

    __device__ static __forceinline__ Site equilibrium(double rho, const Coef& cf)
    {
        Site x;
        const double r2 = rho * rho;
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            if constexpr (has_g(i)) x.s[i] = __builtin_fma(cf.E[i], rho, cf.G[i] * r2);
            else x.s[i] = cf.E[i] * rho;
        });
        return x;
    }

    __device__ static __forceinline__ Site from_f(const double (&f)[Q], const Coef&)
    {
        Site x;
        unroll<Q>([&](auto I) { x.s[I] = f[I]; });
        return x;
    }

    __device__ static __forceinline__ double density(const Site& x)
    {
        double r = x.s[0];
        unroll<Q - 1>([&](auto I) { r = r + x.s[I + 1]; });
        return r;
    }

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
    __device__ static __forceinline__ double pop_g(const char* st, int64_t n, int64_t j, const Coef&)
    {
        return (double)reinterpret_cast<const float*>(st)[I * n + j];
    }

    // density sum and rho^2 term in double, relaxation in single
    __device__ static __forceinline__ void update(const double (&g)[Q], Site& y, const Coef& cf)
    {
        double rho = g[0];
        unroll<Q - 1>([&](auto I) { rho = rho + g[I + 1]; });
        const double r2 = rho * rho;
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            double eq;
            if constexpr (has_g(i)) eq = __builtin_fma(cf.A[i], rho, cf.B[i] * r2);
            else eq = cf.A[i] * rho;
            y.s[i] = __builtin_fmaf(cf.a1mw_f, (float)g[i], (float)eq);
        });
    }

    __device__ static __forceinline__ Site load(const char* st, int64_t n, int64_t j)
    {
        Site x;
        unroll<Q>([&](auto I) { x.s[I] = reinterpret_cast<const float*>(st)[I * n + j]; });
        return x;
    }

    __device__ static __forceinline__ void store(char* st, int64_t n, int64_t j, const Site& x)
    {
        unroll<Q>([&](auto I) { reinterpret_cast<float*>(st)[I * n + j] = x.s[I]; });
    }

    __device__ static __forceinline__ Site equilibrium(double rho, const Coef& cf)
    {
        Site x;
        const double r2 = rho * rho;
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            if constexpr (has_g(i)) x.s[i] = (float)__builtin_fma(cf.E[i], rho, cf.G[i] * r2);
            else x.s[i] = (float)(cf.E[i] * rho);
        });
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
        double r = (double)x.s[0];
        unroll<Q - 1>([&](auto I) { r = r + (double)x.s[I + 1]; });
        return r;
    }

    __device__ static __forceinline__ bool finite(const Site& x)
    {
        bool ok = true;
        unroll<Q>([&](auto I) { ok = ok && __builtin_isfinite(x.s[I]); });
        return ok;
    }
};

// rho in double, non-equilibrium part n_i = S_i - feq_i(rho) in single.
template <int Q>
struct Pol<Q, kSPLIT> {
    struct Site { double rho; float n[Q]; };

    __device__ static __forceinline__ const float* nbase(const char* st, int64_t n)
    {
        return reinterpret_cast<const float*>(st + n * (int64_t)sizeof(double));
    }

    template <int I>
    __device__ static __forceinline__ double eq_of(double rho, const Coef& cf)
    {
        if constexpr (has_g(I)) return __builtin_fma(cf.E[I], rho, cf.G[I] * (rho * rho));
        else return cf.E[I] * rho;
    }

    template <int I>
    __device__ static __forceinline__ double pop(const Site& x, const Coef& cf)
    {
        return eq_of<I>(x.rho, cf) + (double)x.n[I];
    }

    template <int I>
    __device__ static __forceinline__ double pop_g(const char* st, int64_t n, int64_t j, const Coef& cf)
    {
        const double rho = reinterpret_cast<const double*>(st)[j];
        return eq_of<I>(rho, cf) + (double)nbase(st, n)[I * n + j];
    }

    __device__ static __forceinline__ void update(const double (&g)[Q], Site& y, const Coef& cf)
    {
        double rho = g[0];
        unroll<Q - 1>([&](auto I) { rho = rho + g[I + 1]; });
        y.rho = rho;
        unroll<Q>([&](auto I) {
            constexpr int i = I;
            y.n[i] = (float)(cf.a1mw * (g[i] - eq_of<i>(rho, cf)));
        });
    }

    __device__ static __forceinline__ Site load(const char* st, int64_t n, int64_t j)
    {
        Site x;
        x.rho = reinterpret_cast<const double*>(st)[j];
        const float* nb = nbase(st, n);
        unroll<Q>([&](auto I) { x.n[I] = nb[I * n + j]; });
        return x;
    }

    __device__ static __forceinline__ void store(char* st, int64_t n, int64_t j, const Site& x)
    {
        reinterpret_cast<double*>(st)[j] = x.rho;
        float* nb = const_cast<float*>(nbase(st, n));
        unroll<Q>([&](auto I) { nb[I * n + j] = x.n[I]; });
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
        double rho = f[0];
        unroll<Q - 1>([&](auto I) { rho = rho + f[I + 1]; });
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

// ---------------------------------------------------------------- per-site kernels

template <int Q, int P>
__global__ __launch_bounds__(256) void k_init(char* st, int64_t n, const double* __restrict__ rho0, Coef cf)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) PL::store(st, n, j, PL::equilibrium(rho0[j], cf));
}

// One fused pull-stream + density + equilibrium + BGK step per launch (s = 1).
template <int Q, int P>
__global__ __launch_bounds__(256) void k_plain(const char* __restrict__ src, char* __restrict__ dst,
                                               int64_t n, Coef cf)
{
    using PL = Pol<Q, P>;
    constexpr int H = halo_of(Q);
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double g[Q];
    if (j >= H && j + H < n) {
        unroll<Q>([&](auto I) { g[I] = PL::template pop_g<I>(src, n, j - vel(I), cf); });
    } else {
        unroll<Q>([&](auto I) { g[I] = PL::template pop_g<I>(src, n, wrap_site(j - vel(I), n), cf); });
    }
    typename PL::Site y;
    PL::update(g, y, cf);
    PL::store(dst, n, j, y);
}

// ---------------------------------------------------------------- register-resident step engine

template <int Q, int P, int B>
struct Engine {
    using PL = Pol<Q, P>;
    using Site = typename PL::Site;
    static constexpr int H = halo_of(Q);
    static constexpr int NX = nx_of(Q);
    static_assert(B >= H, "a lane must hold at least max|c| sites");

    // write the populations the neighbours pull; column `lane`, row stride ld
    __device__ static __forceinline__ void publish(const Site (&x)[B], double* slot, int ld, int lane,
                                                   const Coef& cf)
    {
        unroll<Q - 1>([&](auto I1) {
            constexpr int i = I1 + 1;
            constexpr int c = vel(i);
            constexpr int k0 = koff(i);
            unroll<iabs(c)>([&](auto T) {
                constexpr int t = T;
                constexpr int src = (c > 0) ? (B - c + t) : t;
                slot[(k0 + t) * ld + lane] = PL::template pop<i>(x[src], cf);
            });
        });
    }

    // one step: registers plus the neighbours' published values
    __device__ static __forceinline__ void step(Site (&x)[B], const double* slot, int ld, int left,
                                                int right, const Coef& cf)
    {
        double hv[NX];
        unroll<Q - 1>([&](auto I1) {
            constexpr int i = I1 + 1;
            constexpr int c = vel(i);
            constexpr int k0 = koff(i);
            unroll<iabs(c)>([&](auto T) {
                constexpr int t = T;
                hv[k0 + t] = slot[(k0 + t) * ld + (c > 0 ? left : right)];
            });
        });
        Site y[B];
        unroll<B>([&](auto Bi) {
            constexpr int b = Bi;
            double g[Q];
            unroll<Q>([&](auto I) {
                constexpr int i = I;
                constexpr int c = vel(i);
                constexpr int sb = b - c;
                if constexpr (sb >= 0 && sb < B) g[i] = PL::template pop<i>(x[sb], cf);
                else if constexpr (c > 0) g[i] = hv[koff(i) + b];
                else g[i] = hv[koff(i) + sb - B];
            });
            PL::update(g, y[b], cf);
        });
        unroll<B>([&](auto Bi) { x[Bi] = y[Bi]; });
    }
};

// Whole periodic lattice of n = B * L sites in one workgroup of L lanes,
// `steps` steps per launch; lane 0 and lane L-1 are neighbours.
template <int Q, int P, int B>
__global__ __launch_bounds__(512) void k_ring(const char* __restrict__ src, char* __restrict__ dst,
                                              int n, int64_t steps, Coef cf)
{
    using E = Engine<Q, P, B>;
    extern __shared__ double xch[];
    const int L = n / B;
    const int lane = threadIdx.x;
    const bool active = lane < L;
    typename E::Site x[B];
    if (active) unroll<B>([&](auto Bi) { x[Bi] = E::PL::load(src, n, (int64_t)lane * B + Bi); });
    const int left = lane == 0 ? L - 1 : lane - 1;
    const int right = lane + 1 >= L ? 0 : lane + 1;
    const int ld = blockDim.x;
    for (int64_t st = 0; st < steps; st++) {
        double* slot = xch + (st & 1) * (E::NX * ld);
        if (active) E::publish(x, slot, ld, lane, cf);
        __syncthreads();
        if (active) E::step(x, slot, ld, left, right, cf);
    }
    if (active) unroll<B>([&](auto Bi) { E::PL::store(dst, n, (int64_t)lane * B + Bi, x[Bi]); });
}

// One halo-widened window of W = B * lanes sites starting at site `ws`
// (periodic modulo n), advanced `s` steps in registers; the `valid` sites from
// ws + H s on are written back.  Sites near the window ends go stale by H per
// step and are never stored.
template <int Q, int P, int B>
__device__ __forceinline__ void window_body(const char* __restrict__ src, char* __restrict__ dst,
                                            int64_t n, int64_t ws, int s, int64_t valid, double* xch,
                                            const Coef& cf)
{
    using E = Engine<Q, P, B>;
    const int L = blockDim.x;
    const int lane = threadIdx.x;
    typename E::Site x[B];
    const int64_t W = (int64_t)L * B;
    const int64_t j0 = ws + (int64_t)lane * B;
    if (ws >= 0 && ws + W <= n) {
        unroll<B>([&](auto Bi) { x[Bi] = E::PL::load(src, n, j0 + Bi); });
    } else {
        unroll<B>([&](auto Bi) { x[Bi] = E::PL::load(src, n, wrap_site(j0 + Bi, n)); });
    }
    const int left = lane == 0 ? L - 1 : lane - 1;
    const int right = lane + 1 == L ? 0 : lane + 1;
    for (int st = 0; st < s; st++) {
        double* slot = xch + (st & 1) * (E::NX * L);
        E::publish(x, slot, L, lane, cf);
        __syncthreads();
        E::step(x, slot, L, left, right, cf);
    }
    const int64_t k_lo = (int64_t)E::H * s;
    unroll<B>([&](auto Bi) {
        const int64_t k = (int64_t)lane * B + Bi;
        if (k >= k_lo && k < k_lo + valid) {
            const int64_t j = ws + k;
            if (j < n) E::PL::store(dst, n, j, x[Bi]);
        }
    });
}

// Large periodic lattice: tile t writes sites [t T, t T + T).
template <int Q, int P, int B>
__global__ __launch_bounds__(256) void k_tile(const char* __restrict__ src, char* __restrict__ dst,
                                              int64_t n, int s, int64_t T, Coef cf)
{
    extern __shared__ double xch[];
    constexpr int H = halo_of(Q);
    const int64_t t0 = (int64_t)blockIdx.x * T;
    window_body<Q, P, B>(src, dst, n, t0 - (int64_t)H * s, s, T, xch, cf);
}

// Ensemble: one window per workgroup from a descriptor table.
template <int Q, int P, int B>
__global__ __launch_bounds__(256) void k_ens(char* base, const WinDesc* __restrict__ desc, Coef cf)
{
    extern __shared__ double xch[];
    const WinDesc d = desc[blockIdx.x];
    window_body<Q, P, B>(base + d.src_off, base + d.dst_off, d.n, d.start, d.steps, d.valid, xch, cf);
}

// ---------------------------------------------------------------- readout and diagnostics

template <int Q, int P>
__global__ __launch_bounds__(256) void k_read_rho(const char* __restrict__ st, int64_t n, double* __restrict__ out)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) out[j] = PL::density(PL::load(st, n, j));
}

template <int Q, int P>
__global__ __launch_bounds__(256) void k_read_f(const char* __restrict__ st, int64_t n, double* __restrict__ out,
                                                int pre, Coef cf)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    unroll<Q>([&](auto I) {
        const int64_t s = pre ? wrap_site(j - vel(I), n) : j;
        out[I * n + j] = PL::template pop_g<I>(st, n, s, cf);
    });
}

template <int Q, int P>
__global__ __launch_bounds__(256) void k_write_f(char* st, int64_t n, const double* __restrict__ in, Coef cf)
{
    using PL = Pol<Q, P>;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double f[Q];
    unroll<Q>([&](auto I) { f[I] = in[I * n + j]; });
    PL::store(st, n, j, PL::from_f(f, cf));
}

__global__ void k_zero_int(int* p) { *p = 0; }

constexpr int kDiagBlocks = 256;

// Stage 1: block b sums the densities of sites b*256 + t + k*65536 (fixed
// order), then a fixed tree over its 256 threads.
template <int Q, int P>
__global__ __launch_bounds__(256) void k_diag1(const char* __restrict__ st, int64_t n, double* partial, int* flag)
{
    using PL = Pol<Q, P>;
    __shared__ double red[256];
    double acc = 0.0;
    bool ok = true;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)kDiagBlocks * 256) {
        const auto x = PL::load(st, n, j);
        acc += PL::density(x);
        ok = ok && PL::finite(x);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
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
            else { constexpr int Q_ = 5, P_ = kSPLIT; CALL; }             \
        } else {                                                         \
            if ((prec) == kFP64) { constexpr int Q_ = 7, P_ = kFP64; CALL; } \
            else if ((prec) == kFP32) { constexpr int Q_ = 7, P_ = kFP32; CALL; } \
            else { constexpr int Q_ = 7, P_ = kSPLIT; CALL; }             \
        }                                                                \
    } while (0)

size_t state_copy_bytes(int64_t n, int q, int prec)
{
    size_t b;
    if (prec == kFP64) b = (size_t)q * (size_t)n * 8;
    else if (prec == kFP32) b = (size_t)q * (size_t)n * 4;
    else b = (size_t)n * 8 + (size_t)q * (size_t)n * 4;
    return (b + 255) & ~(size_t)255;
}

int max_lds_bytes()
{
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            cached = v;
        else
            cached = 65536;
    }
    return cached;
}

int ring_lds_bytes(int q, int lanes) { return 2 * nx_of(q) * lanes * (int)sizeof(double); }

template <class K>
static int prep_lds(K kernel, int bytes)
{
    if (bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return (int)e;
    }
    return 0;
}

int launch_init(int q, int prec, void* state, int64_t n, const double* rho0, const Coef& cf, void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_init<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (char*)state, n, rho0, cf)));
    return (int)hipGetLastError();
}

int launch_plain(int q, int prec, const void* src, void* dst, int64_t n, const Coef& cf, void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_plain<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (const char*)src, (char*)dst, n, cf)));
    return (int)hipGetLastError();
}

template <int Q, int P, int B>
static int ring_one(const void* src, void* dst, int64_t n, int64_t steps, const Coef& cf, void* stream)
{
    const int L = (int)(n / B);
    const int lanes = ((L + 63) / 64) * 64;
    const int lds = ring_lds_bytes(Q, lanes);
    int e = prep_lds(k_ring<Q, P, B>, lds);
    if (e) return e;
    k_ring<Q, P, B><<<1, lanes, lds, (hipStream_t)stream>>>((const char*)src, (char*)dst, (int)n, steps, cf);
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
static int tile_one(const void* src, void* dst, int64_t n, int s, int lanes, const Coef& cf, void* stream)
{
    const int64_t W = (int64_t)lanes * B;
    const int64_t T = W - 2 * (int64_t)halo_of(Q) * s;
    if (T <= 0) return (int)hipErrorInvalidValue;
    const int64_t tiles = (n + T - 1) / T;
    const int lds = ring_lds_bytes(Q, lanes);
    int e = prep_lds(k_tile<Q, P, B>, lds);
    if (e) return e;
    k_tile<Q, P, B><<<(unsigned)tiles, lanes, lds, (hipStream_t)stream>>>((const char*)src, (char*)dst, n, s, T, cf);
    return (int)hipGetLastError();
}

int launch_tile(int q, int prec, int B, int lanes, const void* src, void* dst, int64_t n, int s,
                const Coef& cf, void* stream)
{
    if (lanes <= 0 || lanes > 256 || lanes % 64) return (int)hipErrorInvalidValue;
    if (B == 4) { KSLB_DISPATCH_QP(q, prec, return (tile_one<Q_, P_, 4>(src, dst, n, s, lanes, cf, stream))); }
    if (B == 8) { KSLB_DISPATCH_QP(q, prec, return (tile_one<Q_, P_, 8>(src, dst, n, s, lanes, cf, stream))); }
    return (int)hipErrorInvalidValue;
}

template <int Q, int P, int B>
static int ens_one(char* base, const WinDesc* desc, int nwin, int lanes, const Coef& cf, void* stream)
{
    const int lds = ring_lds_bytes(Q, lanes);
    int e = prep_lds(k_ens<Q, P, B>, lds);
    if (e) return e;
    k_ens<Q, P, B><<<(unsigned)nwin, lanes, lds, (hipStream_t)stream>>>(base, desc, cf);
    return (int)hipGetLastError();
}

int launch_ens(int q, int prec, int B, int lanes, char* base, const WinDesc* desc, int nwin,
               const Coef& cf, void* stream)
{
    if (nwin <= 0) return 0;
    if (lanes <= 0 || lanes > 256 || lanes % 64) return (int)hipErrorInvalidValue;
    if (B == 4) { KSLB_DISPATCH_QP(q, prec, return (ens_one<Q_, P_, 4>(base, desc, nwin, lanes, cf, stream))); }
    if (B == 8) { KSLB_DISPATCH_QP(q, prec, return (ens_one<Q_, P_, 8>(base, desc, nwin, lanes, cf, stream))); }
    return (int)hipErrorInvalidValue;
}

int launch_read_rho(int q, int prec, const void* state, int64_t n, double* out, void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_read_rho<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (const char*)state, n, out)));
    return (int)hipGetLastError();
}

int launch_read_f(int q, int prec, const void* state, int64_t n, double* out, int pre, const Coef& cf,
                  void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_read_f<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (const char*)state, n, out, pre, cf)));
    return (int)hipGetLastError();
}

int launch_write_f(int q, int prec, void* state, int64_t n, const double* in, const Coef& cf, void* stream)
{
    KSLB_DISPATCH_QP(q, prec, (k_write_f<Q_, P_><<<blocks_for(n), 256, 0, (hipStream_t)stream>>>(
                                  (char*)state, n, in, cf)));
    return (int)hipGetLastError();
}

int launch_diag(int q, int prec, const void* state, int64_t n, double* partial, int* flag, double* mass_out,
                void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    k_zero_int<<<1, 1, 0, s>>>(flag);
    KSLB_DISPATCH_QP(q, prec, (k_diag1<Q_, P_><<<kDiagBlocks, 256, 0, s>>>((const char*)state, n, partial, flag)));
    k_diag2<<<1, 1, 0, s>>>(partial, mass_out);
    return (int)hipGetLastError();
}

}  // namespace kslb
