// kslb_api.cpp -- C ABI of libkslb (see include/kslb.h).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/kslb.h"
#include "kslb_internal.h"

using namespace kslb;

namespace {

thread_local std::string g_err;

kslb_status fail(kslb_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

kslb_status hip_fail(int e, const char* what)
{
    return fail(KSLB_EDEVICE, "%s: %s", what, hipGetErrorString((hipError_t)e));
}

// Make the object's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Diagnostics area at the end of a lattice's (or ensemble's) buffer: 256
// partial sums, the mass, the non-finite flag and, from kCtlOffset, the
// control words of the multi-workgroup kernel.
constexpr size_t kDiagBytes = 4096;
constexpr size_t kCtlOffset = 2304;

bool valid_shape(int64_t n, int q, int prec)
{
    return n > 0 && n < (int64_t(1) << 40) && (q == 5 || q == 7) && prec >= 0 && prec <= 3;
}

int halo(int q) { return q == 5 ? 2 : 3; }

void fold(Coef& cf, const double* E, const double* G, double omega, int q)
{
    std::memset(&cf, 0, sizeof cf);
    for (int i = 0; i < q; i++) {
        cf.E[i] = E[i];
        cf.G[i] = G[i];
        cf.A[i] = omega * E[i];
        cf.B[i] = omega * G[i];
    }
    cf.a1mw = 1.0 - omega;
    cf.a1mw_f = (float)cf.a1mw;
}

// Coefficients + tau policy shared by lattices and ensembles.
struct Physics {
    bool set = false;
    double E[7] = {}, G[7] = {}, jkm[5] = {};
    double tau = 0.0, omega = 0.0;
    Coef cf{};
};

kslb_status set_physics(Physics& ph, int q, double dX, double dT, double tau, int dm_variant,
                        int guard_policy, double rho_max)
{
    if (!(dX > 0.0) || !(dT > 0.0) || !std::isfinite(dX) || !std::isfinite(dT))
        return fail(KSLB_EINVAL, "dX and dT must be positive and finite");
    if (dm_variant != KSLB_DM_DERIVED && dm_variant != KSLB_DM_LITERAL)
        return fail(KSLB_EINVAL, "bad dm_variant %d", dm_variant);
    if (guard_policy < KSLB_GUARD_REFUSE || guard_policy > KSLB_GUARD_OFF)
        return fail(KSLB_EINVAL, "bad guard_policy %d", guard_policy);
    if (!(rho_max >= 0.0) || !std::isfinite(rho_max)) return fail(KSLB_EINVAL, "rho_max must be >= 0");
    if (tau <= 0.0) tau = tau_fit(q, dX, dT);
    if (!(tau >= kTauMin) || !std::isfinite(tau))
        return fail(KSLB_EINVAL, "tau = %g is below %g (M has a pole near 0.908)", tau, kTauMin);
    double E[7], G[7], jkm[5];
    for (int tries = 0;; tries++) {
        if (scheme_coefficients(q, dX, dT, tau, dm_variant, jkm, E, G))
            return fail(KSLB_EINVAL, "coefficients undefined for these parameters");
        if (guard_policy == KSLB_GUARD_OFF) break;
        if (stability_check(q, E, G, 1.0 / tau, dX, dT, rho_max)) break;
        if (guard_policy == KSLB_GUARD_REFUSE)
            return fail(KSLB_EUNSTABLE, "linearly unstable at dX=%g dT=%g tau=%.6f (q=%d)", dX, dT, tau, q);
        if (tries >= 200)
            return fail(KSLB_EUNSTABLE, "no stable tau found up to %.3f", tau);
        tau += 0.02;
    }
    ph.set = true;
    std::memcpy(ph.E, E, sizeof E);
    std::memcpy(ph.G, G, sizeof G);
    std::memcpy(ph.jkm, jkm, sizeof jkm);
    ph.tau = tau;
    ph.omega = 1.0 / tau;
    fold(ph.cf, E, G, ph.omega, q);
    return KSLB_OK;
}

kslb_status rho_mode_check(int prec, const Physics& ph)
{
    if (prec == kRHO && ph.omega != 1.0)
        return fail(KSLB_EINVAL, "the rho-only storage needs tau = 1 exactly (got tau = %.17g)", ph.tau);
    return KSLB_OK;
}

}  // namespace

// ============================================================================
// lattice
// ============================================================================

struct kslb_lattice {
    int64_t n = 0;
    int q = 0, prec = 0, device = 0;
    char* buf = nullptr;
    size_t bytes = 0, copy = 0;
    hipStream_t stream = nullptr;
    int cur = 0;                       // which ping-pong copy holds the state
    bool have_state = false;
    Physics ph;
    int kernel = KSLB_KERNEL_AUTO;
    int tile_steps = 0;
    int64_t step = 0;
    double* staging = nullptr;         // Q x n doubles, only for host transfers
    char* span_scratch = nullptr;      // edge slots of the multi-workgroup kernel
    size_t span_bytes = 0;
    bool ctl_ready = false;            // control words set up (first multi-workgroup advance)
    bool fixed = false;                // fixed-end boundary (Table 3 problem)
    Ends ends{0.0, 0.0};

    char* state() { return buf + (size_t)cur * copy; }
    char* other() { return buf + (size_t)(1 - cur) * copy; }
    double* diag() { return reinterpret_cast<double*>(buf + 2 * copy); }
    int* ctl() { return reinterpret_cast<int*>(buf + 2 * copy + kCtlOffset); }
    const int* sticky() { return ctl_ready ? ctl() + span_ctl_error_index() : nullptr; }
};

namespace {

kslb_status ensure_staging(kslb_lattice* L)
{
    if (L->staging) return KSLB_OK;
    void* p = nullptr;
    int e = hipMalloc(&p, sizeof(double) * (size_t)L->q * (size_t)L->n);
    if (e) return fail(KSLB_ENOMEM, "staging allocation of %zu bytes failed",
                       sizeof(double) * (size_t)L->q * (size_t)L->n);
    L->staging = (double*)p;
    return KSLB_OK;
}

// ring kernel: B in {8, 4} dividing n, at most ring_max_lanes() lanes, and
// the exchange area in LDS
int ring_sites_per_lane(int64_t n, int q, int lds_bytes)
{
    if (ring_lds_bytes(q) > lds_bytes) return 0;
    const int Bs[2] = {8, 4};
    for (int B : Bs) {
        if (n % B) continue;
        const int64_t L = n / B;
        if (L < 1 || L > ring_max_lanes()) continue;
        return B;
    }
    return 0;
}


// Device limits a plan assumes: SPAN owners that may run at once, and the
// dynamic LDS one workgroup may use.
struct Limits {
    int64_t span_owners;
    int lds_bytes;
};

// Every SPAN owner spins on its neighbours' edges, so all of a launch's
// owners must be resident together.  A plan takes at most half of what the
// device keeps resident (one owner per SIMD where the occupancy allows two),
// leaving room for other work on the device, and never more than this.
constexpr int64_t kSpanMaxOwners = 2048;

Limits device_limits(int q, int prec, bool fixed)
{
    return Limits{std::min<int64_t>(kSpanMaxOwners, span_device_owners(q, prec, fixed) / 2), max_lds_bytes()};
}

// Multi-workgroup plan: nwg single-wave owners of about n / nwg sites each,
// every window (own sites + 2 H s halo, a halo possibly spanning several
// owners) within span_lanes() x span_sites_per_lane(q, prec) slots.  Returns
// nwg, or 0 when the shape cannot use it or needs more than max_owners owners.
int span_plan(int64_t n, int q, int prec, int s, int64_t max_owners)
{
    const int64_t W = (int64_t)span_lanes() * span_sites_per_lane(q, prec);
    const int64_t hs = (int64_t)halo(q) * s;
    const int64_t own = W - 2 * hs;
    if (s < 1 || own < 1) return 0;
    const int64_t nwg = (n + own - 1) / own;
    if (nwg < 2 || nwg > std::min(max_owners, kSpanMaxOwners)) return 0;
    return (int)nwg;
}

// Default steps between edge exchanges: the largest s that plans with each
// owner's own sites at least 2/3 of the halo depth (3 W >= 8 H s).  Longer
// intervals mean more, thinner owners whose halos gather from many slots;
// measured on D1Q7 N = 4096: s = 21, 24, 28, 31 (63, 86, 171, 683 owners) ran
// 26.7, 25.1, 26.1, 57 ms per 10^5 steps; s = 22, 23, 25, 26, 27 ran 26.7,
// 26.3, 26.2, 26.4, 26.6 ms.
int span_default_steps(int64_t n, int q, int prec, int64_t max_owners)
{
    const int64_t W = (int64_t)span_lanes() * span_sites_per_lane(q, prec);
    for (int s = (int)((3 * W) / (8 * halo(q))); s >= 1; s--)
        if (span_plan(n, q, prec, s, max_owners)) return s;
    return 0;
}

// Device scratch of the SPAN kernel: the edge slots of one launch, at most
// kSpanSlotBytes of them (a longer advance is split into launches of
// (slots + 1) s steps).  Its control words live in the lattice's own buffer.
constexpr size_t kSpanSlotBytes = size_t(256) << 20;

// AUTO: one lattice small enough for a few hundred single-wave owners runs
// on SPAN, provided its owners fit the device with an exchange at most every
// kSpanAutoMinSteps steps (shorter intervals spend most of a launch waiting on
// exchanges); otherwise RESIDENT when it fits one workgroup, else TILED.
constexpr int64_t kSpanAutoMaxSites = 65536;
constexpr int kSpanAutoMinSteps = 12;

// Steps per tiled launch, even so that every lane's first site is even (its
// vector accesses).  Longer launches re-read the state less often but
// recompute a wider halo (2 H s of the window's W sites).  Sweeps of s on
// N = 2^24 put the optimum at 80 for D1Q7 FP64 (1063 GLUPS; 1060 at 64,
// 1063 at 96), 112 for D1Q5 FP64 (1447; 1396 at 64), 64 for the rho-only
// D1Q7 state (1931; 1925 at 96, 1913 at 128), 128 for rho-only D1Q5 (2371;
// 2325 at 64), 48 for FP32 (D1Q7 975-981, 931 at 64, 912 at 80; D1Q5
// 1302-1311, 1293 at 64) and for split 32 on D1Q7 (563, 555 at 40, 531 at
// 64) and 40 on D1Q5 (817, 792 at 64).
int default_tile_steps(int q, int prec)
{
    if (prec == kFP64) return q == 7 ? 80 : 112;
    if (prec == kRHO) return q == 7 ? 64 : 128;
    if (prec == kFP32) return 48;
    return q == 7 ? 32 : 40;
}

kslb_status check_lat(const kslb_lattice* L)
{
    if (!L) return fail(KSLB_EINVAL, "null lattice");
    return KSLB_OK;
}

// Longest advance one launch of the RESIDENT or SPAN kernel covers.
constexpr int64_t kMaxStepsPerLaunch = int64_t(1) << 20;

// The kernel class an advance of this lattice runs (AUTO resolved) and its
// step parameter: steps per launch for TILED, steps between edge exchanges
// for SPAN, 0 otherwise.  kernel = AUTO on return means no class fits.
struct KernelChoice {
    int kernel;
    int steps;
};

// The kernel class an advance runs for this shape, boundary and request
// (AUTO resolved) under the device limits lim, with its step parameter.
// AUTO takes SPAN only when all its owners fit lim.span_owners.
KernelChoice plan_kernel(int64_t n, int q, int prec, bool fixed, int req, int req_steps, const Limits& lim)
{
    int kernel = req;
    if (kernel == KSLB_KERNEL_AUTO) {
        if (n <= kSpanAutoMaxSites && span_default_steps(n, q, prec, lim.span_owners) >= kSpanAutoMinSteps)
            kernel = KSLB_KERNEL_SPAN;
        else if (fixed) kernel = KSLB_KERNEL_PLAIN;
        else kernel = ring_sites_per_lane(n, q, lim.lds_bytes) ? KSLB_KERNEL_RESIDENT : KSLB_KERNEL_TILED;
    }
    int steps = 0;
    if (kernel == KSLB_KERNEL_SPAN)
        steps = (req == KSLB_KERNEL_SPAN && req_steps > 0) ? req_steps : span_default_steps(n, q, prec, lim.span_owners);
    else if (kernel == KSLB_KERNEL_TILED)
        steps = req_steps > 0 ? req_steps : default_tile_steps(q, prec);
    return KernelChoice{kernel, steps};
}

}  // namespace

namespace {

// Edge slots one SPAN launch can use (within slot_bytes), and the steps such
// a launch covers.
int64_t span_slot_capacity(int64_t per_exchange, int s, size_t slot_bytes)
{
    return std::max<int64_t>(1, std::min<int64_t>((int64_t)slot_bytes / per_exchange, kMaxStepsPerLaunch / s));
}

int64_t span_steps_per_launch(int64_t per_exchange, int s, size_t slot_bytes)
{
    return std::min<int64_t>(kMaxStepsPerLaunch, (span_slot_capacity(per_exchange, s, slot_bytes) + 1) * s);
}

// Control words of the multi-workgroup kernel, in the lattice's buffer: set
// up once, before its first multi-workgroup launch.
kslb_status span_ctl_setup(kslb_lattice* L)
{
    if (L->ctl_ready) return KSLB_OK;
    int e = launch_span_ctl_init(L->ctl(), span_ctl_ints(), L->stream);
    if (e) return hip_fail(e, "SPAN control init");
    L->ctl_ready = true;
    return KSLB_OK;
}

// Edge slots for a SPAN advance of n_steps from the library's exchange area:
// those of (up to) one launch; *slots_out is every slot the area holds in
// this geometry.  Each launch refills the slots it uses with the sentinel.
kslb_status span_prepare(kslb_lattice* L, int64_t per, int s, int64_t n_steps, int64_t* slots_out)
{
    const int64_t exchanges = (std::min(n_steps, span_steps_per_launch(per, s, kSpanSlotBytes)) + s - 1) / s - 1;
    const int64_t want = std::max<int64_t>(1, std::min(span_slot_capacity(per, s, kSpanSlotBytes), exchanges));
    int64_t have = L->span_scratch ? (int64_t)L->span_bytes / per : 0;
    if (have < want) {
        if (L->span_scratch) {
            int e = hipStreamSynchronize(L->stream);   // earlier launches may still read the slots
            if (e) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(L->span_scratch);
            L->span_scratch = nullptr;
            L->span_bytes = 0;
        }
        const size_t need = (size_t)want * (size_t)per;
        void* p = nullptr;
        if (hipMalloc(&p, need)) return fail(KSLB_ENOMEM, "exchange area of %zu bytes failed", need);
        L->span_scratch = (char*)p;
        L->span_bytes = need;
        have = want;
    }
    *slots_out = have;
    return KSLB_OK;
}

// A new state: forget SPAN timeouts of the previous one.
kslb_status span_clear_error(kslb_lattice* L)
{
    if (!L->ctl_ready) return KSLB_OK;
    int e = launch_span_set_ctl(L->ctl(), span_ctl_error_index(), 0, L->stream);
    return e ? hip_fail(e, "SPAN control") : KSLB_OK;
}

// After a synchronising transfer: EDEVICE while the sticky error word is set
// (a SPAN launch stopped early and the state is not valid).  Synchronises.
kslb_status span_check_error(kslb_lattice* L)
{
    if (!L->ctl_ready) return KSLB_OK;
    int err = 0;
    int e = hipMemcpyAsync(&err, L->ctl() + span_ctl_error_index(), sizeof err, hipMemcpyDeviceToHost, L->stream);
    if (!e) e = hipStreamSynchronize(L->stream);
    if (e) return hip_fail(e, "SPAN control copy");
    if (err)
        return fail(KSLB_EDEVICE, "a multi-workgroup launch stopped early (a neighbour's edge never arrived or "
                                  "the launch was aborted); the state is not valid until it is replaced");
    return KSLB_OK;
}

}  // namespace

extern "C" {

kslb_status kslb_scheme_coefficients(int q, double dX, double dT, double tau, int dm_variant,
                                     double* jkm, double* E, double* G)
{
    if (!jkm) return fail(KSLB_EINVAL, "jkm must not be NULL");
    if (scheme_coefficients(q, dX, dT, tau, dm_variant, jkm, E, G))
        return fail(KSLB_EINVAL, "bad scheme parameters (q=%d dX=%g dT=%g tau=%g)", q, dX, dT, tau);
    return KSLB_OK;
}

double kslb_tau_fit(int q, double dX, double dT) { return tau_fit(q, dX, dT); }

kslb_status kslb_spectral_radius(int q, const double* E, const double* G, double omega, double rho_bar,
                                 double k, double* radius)
{
    if ((q != 5 && q != 7) || !E || !G || !radius) return fail(KSLB_EINVAL, "bad arguments");
    *radius = spectral_radius(q, E, G, omega, rho_bar, k);
    return KSLB_OK;
}

kslb_status kslb_stability_check(int q, const double* E, const double* G, double omega, double dX,
                                 double dT, double rho_max, int* stable)
{
    if ((q != 5 && q != 7) || !E || !G || !stable || !(dX > 0) || !(dT > 0))
        return fail(KSLB_EINVAL, "bad arguments");
    *stable = stability_check(q, E, G, omega, dX, dT, rho_max);
    return KSLB_OK;
}

size_t kslb_state_bytes(int64_t n_sites, int q, int precision)
{
    if (!valid_shape(n_sites, q, precision)) return 0;
    return 2 * state_copy_bytes(n_sites, q, precision) + kDiagBytes;
}

kslb_status kslb_create(kslb_lattice** out, int64_t n_sites, int q, int precision, void* dev_buf,
                        size_t buf_bytes, void* hip_stream)
{
    if (!out) return fail(KSLB_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!valid_shape(n_sites, q, precision))
        return fail(KSLB_EINVAL, "bad shape n=%lld q=%d precision=%d", (long long)n_sites, q, precision);
    if (!dev_buf) return fail(KSLB_EINVAL, "null device buffer");
    if (reinterpret_cast<uintptr_t>(dev_buf) % 256) return fail(KSLB_EINVAL, "buffer not 256-byte aligned");
    const size_t need = kslb_state_bytes(n_sites, q, precision);
    if (buf_bytes < need) return fail(KSLB_ENOMEM, "buffer has %zu bytes, needs %zu", buf_bytes, need);
    int dev = 0;
    int e = hipGetDevice(&dev);
    if (e) return hip_fail(e, "hipGetDevice");
    kslb_lattice* L = new (std::nothrow) kslb_lattice;
    if (!L) return fail(KSLB_ENOMEM, "host allocation failed");
    L->n = n_sites;
    L->q = q;
    L->prec = precision;
    L->device = dev;
    L->buf = (char*)dev_buf;
    L->bytes = buf_bytes;
    L->copy = state_copy_bytes(n_sites, q, precision);
    L->stream = (hipStream_t)hip_stream;
    *out = L;
    return KSLB_OK;
}

kslb_status kslb_set_physical(kslb_lattice* L, double dX, double dT, double tau, int dm_variant,
                              int guard_policy, double rho_max)
{
    if (auto s = check_lat(L)) return s;
    Physics ph;
    kslb_status st = set_physics(ph, L->q, dX, dT, tau, dm_variant, guard_policy, rho_max);
    if (st) return st;
    if ((st = rho_mode_check(L->prec, ph))) return st;
    L->ph = ph;
    return KSLB_OK;
}

kslb_status kslb_set_coefficients(kslb_lattice* L, const double* E, const double* G, double omega)
{
    if (auto s = check_lat(L)) return s;
    if (!E || !G) return fail(KSLB_EINVAL, "E and G must not be NULL");
    if (!(omega > 0.0 && omega < 2.0)) return fail(KSLB_EINVAL, "omega must lie in (0, 2)");
    for (int i = 0; i < L->q; i++) {
        if (!std::isfinite(E[i]) || !std::isfinite(G[i])) return fail(KSLB_EINVAL, "non-finite coefficient");
        const bool g_allowed = (i >= 1 && i <= 4);
        if (!g_allowed && G[i] != 0.0) return fail(KSLB_EINVAL, "G_%d must be 0 (c = 0 or +-3)", i);
    }
    for (int k = 1; 2 * k < L->q; k++)
        if (E[2 * k] != E[2 * k - 1] || G[2 * k] != -G[2 * k - 1])
            return fail(KSLB_EINVAL, "E must be even and G odd in c (E_%d = E_%d, G_%d = -G_%d)", 2 * k, 2 * k - 1,
                        2 * k, 2 * k - 1);
    Physics ph;
    ph.set = true;
    for (int i = 0; i < L->q; i++) { ph.E[i] = E[i]; ph.G[i] = G[i]; }
    ph.omega = omega;
    ph.tau = 1.0 / omega;
    fold(ph.cf, ph.E, ph.G, omega, L->q);
    if (auto st = rho_mode_check(L->prec, ph)) return st;
    L->ph = ph;
    return KSLB_OK;
}

kslb_status kslb_get_coefficients(const kslb_lattice* L, double* E, double* G, double* omega, double* tau,
                                  double* jkm)
{
    if (auto s = check_lat(L)) return s;
    if (!L->ph.set) return fail(KSLB_ESTATE, "coefficients not set");
    for (int i = 0; i < L->q; i++) {
        if (E) E[i] = L->ph.E[i];
        if (G) G[i] = L->ph.G[i];
    }
    if (omega) *omega = L->ph.omega;
    if (tau) *tau = L->ph.tau;
    if (jkm) std::memcpy(jkm, L->ph.jkm, sizeof L->ph.jkm);
    return KSLB_OK;
}

kslb_status kslb_set_kernel(kslb_lattice* L, int kernel, int steps_per_launch)
{
    if (auto s = check_lat(L)) return s;
    if (kernel < KSLB_KERNEL_AUTO || kernel > KSLB_KERNEL_SPAN) return fail(KSLB_EINVAL, "bad kernel %d", kernel);
    if (steps_per_launch < 0) return fail(KSLB_EINVAL, "steps_per_launch must be >= 0");
    if (kernel == KSLB_KERNEL_RESIDENT || kernel == KSLB_KERNEL_SPAN) {
        DeviceGuard g(L->device);
        const Limits lim = device_limits(L->q, L->prec, L->fixed);
        if (kernel == KSLB_KERNEL_RESIDENT && !ring_sites_per_lane(L->n, L->q, lim.lds_bytes))
            return fail(KSLB_EINVAL, "n=%lld cannot use the resident kernel (needs n = B*L, B in {4,8}, L <= 512)",
                        (long long)L->n);
        if (kernel == KSLB_KERNEL_SPAN) {
            const int sp = steps_per_launch > 0 ? steps_per_launch : span_default_steps(L->n, L->q, L->prec, lim.span_owners);
            if (!sp || !span_plan(L->n, L->q, L->prec, sp, lim.span_owners))
                return fail(KSLB_EINVAL,
                            "n=%lld cannot be split over at most %lld resident workgroups with %d steps between "
                            "exchanges", (long long)L->n, (long long)lim.span_owners, sp);
        }
    }
    if (kernel == KSLB_KERNEL_TILED && steps_per_launch > 0) {
        if (tile_lanes() * tile_sites_per_lane(L->prec) - 2 * halo(L->q) * steps_per_launch <= 0)
            return fail(KSLB_EINVAL, "steps_per_launch %d leaves no valid sites in a tile", steps_per_launch);
    }
    L->kernel = kernel;
    L->tile_steps = steps_per_launch;
    return KSLB_OK;
}

}  // extern "C"

namespace {

// Launch shape of a planned class: the most steps one launch advances, the
// steps between edge exchanges (SPAN), the workgroups of one launch and the
// lanes of each.
void describe(const KernelChoice& kc, int64_t n, int q, int prec, const Limits& lim, int* kernel,
              int* steps_per_launch, int* exchange_steps, int64_t* workgroups, int* lanes_per_workgroup)
{
    int per_launch = 1, exch = 0, lanes = 256;
    int64_t wg = (n + 255) / 256;
    switch (kc.kernel) {
    case KSLB_KERNEL_RESIDENT: {
        const int rb = ring_sites_per_lane(n, q, lim.lds_bytes);
        per_launch = (int)kMaxStepsPerLaunch;
        wg = 1;
        lanes = rb ? (int)(n / rb) : 0;
        break;
    }
    case KSLB_KERNEL_SPAN:
        exch = kc.steps;
        wg = kc.steps ? span_plan(n, q, prec, kc.steps, lim.span_owners) : 0;
        per_launch = wg ? (int)span_steps_per_launch(wg * span_edge_copy_bytes(q, prec, n, (int)wg, kc.steps),
                                                     kc.steps, kSpanSlotBytes)
                        : 0;
        lanes = span_lanes();
        break;
    case KSLB_KERNEL_TILED: {
        per_launch = kc.steps;
        const int64_t T = (int64_t)tile_lanes() * tile_sites_per_lane(prec) - 2 * (int64_t)halo(q) * kc.steps;
        wg = T > 0 ? (n + T - 1) / T : 0;
        break;
    }
    default:
        break;
    }
    if (kernel) *kernel = kc.kernel;
    if (steps_per_launch) *steps_per_launch = per_launch;
    if (exchange_steps) *exchange_steps = exch;
    if (workgroups) *workgroups = wg;
    if (lanes_per_workgroup) *lanes_per_workgroup = lanes;
}

}  // namespace

extern "C" {

kslb_status kslb_get_kernel(const kslb_lattice* L, int* kernel, int* steps_per_launch, int* exchange_steps,
                            int64_t* workgroups, int* lanes_per_workgroup)
{
    if (auto s = check_lat(L)) return s;
    DeviceGuard g(L->device);
    const Limits lim = device_limits(L->q, L->prec, L->fixed);
    const KernelChoice kc = plan_kernel(L->n, L->q, L->prec, L->fixed, L->kernel, L->tile_steps, lim);
    describe(kc, L->n, L->q, L->prec, lim, kernel, steps_per_launch, exchange_steps, workgroups,
             lanes_per_workgroup);
    return KSLB_OK;
}

kslb_status kslb_plan_kernel(int64_t n_sites, int q, int precision, int boundary, int kernel, int steps_per_launch,
                             int64_t span_owners, int lds_bytes, int* kernel_out, int* steps_per_launch_out,
                             int* exchange_steps, int64_t* workgroups, int* lanes_per_workgroup)
{
    if (!valid_shape(n_sites, q, precision)) return fail(KSLB_EINVAL, "bad shape");
    if (kernel < KSLB_KERNEL_AUTO || kernel > KSLB_KERNEL_SPAN) return fail(KSLB_EINVAL, "bad kernel %d", kernel);
    if (boundary != KSLB_PERIODIC && boundary != KSLB_FIXED_ENDS) return fail(KSLB_EINVAL, "bad boundary %d", boundary);
    if (steps_per_launch < 0 || span_owners < 0 || lds_bytes < 0) return fail(KSLB_EINVAL, "negative argument");
    const bool fixed = boundary == KSLB_FIXED_ENDS;
    Limits lim{std::min(kSpanMaxOwners, span_owners / 2), lds_bytes};
    if (span_owners == 0 || lds_bytes == 0) {
        const Limits dev = device_limits(q, precision, fixed);
        if (span_owners == 0) lim.span_owners = dev.span_owners;
        if (lds_bytes == 0) lim.lds_bytes = dev.lds_bytes;
    }
    const KernelChoice kc = plan_kernel(n_sites, q, precision, fixed, kernel, steps_per_launch, lim);
    if (kc.kernel == KSLB_KERNEL_SPAN && !span_plan(n_sites, q, precision, kc.steps, lim.span_owners))
        return fail(KSLB_EINVAL, "n=%lld cannot be split over at most %lld resident workgroups", (long long)n_sites,
                    (long long)lim.span_owners);
    if (kc.kernel == KSLB_KERNEL_RESIDENT && !ring_sites_per_lane(n_sites, q, lim.lds_bytes))
        return fail(KSLB_EINVAL, "n=%lld cannot use the resident kernel", (long long)n_sites);
    if (fixed && kc.kernel != KSLB_KERNEL_PLAIN && kc.kernel != KSLB_KERNEL_SPAN)
        return fail(KSLB_EINVAL, "fixed ends run on the PLAIN and SPAN kernels only");
    describe(kc, n_sites, q, precision, lim, kernel_out, steps_per_launch_out, exchange_steps, workgroups,
             lanes_per_workgroup);
    return KSLB_OK;
}

kslb_status kslb_set_boundary(kslb_lattice* L, int mode, double rho_left, double rho_right)
{
    if (auto s = check_lat(L)) return s;
    if (mode == KSLB_PERIODIC) {
        L->fixed = false;
        return KSLB_OK;
    }
    if (mode != KSLB_FIXED_ENDS) return fail(KSLB_EINVAL, "bad boundary mode %d", mode);
    if (!std::isfinite(rho_left) || !std::isfinite(rho_right)) return fail(KSLB_EINVAL, "non-finite end value");
    if (L->n < 3) return fail(KSLB_EINVAL, "fixed ends need at least 3 sites");
    L->fixed = true;
    L->ends = Ends{rho_left, rho_right};
    return KSLB_OK;
}

kslb_status kslb_init_rho(kslb_lattice* L, const double* rho, int rho_on_device)
{
    if (auto s = check_lat(L)) return s;
    if (!rho) return fail(KSLB_EINVAL, "rho must not be NULL");
    if (!L->ph.set) return fail(KSLB_ESTATE, "set the coefficients before init_rho");
    DeviceGuard g(L->device);
    const double* src = rho;
    if (!rho_on_device) {
        if (auto s = ensure_staging(L)) return s;
        int e = hipMemcpyAsync(L->staging, rho, sizeof(double) * (size_t)L->n, hipMemcpyHostToDevice, L->stream);
        if (e) return hip_fail(e, "hipMemcpyAsync(rho)");
        src = L->staging;
    }
    L->cur = 0;
    int e = L->fixed ? launch_init_fixed(L->q, L->prec, L->state(), L->n, src, L->ph.cf, L->ends, L->stream)
                     : launch_init(L->q, L->prec, L->state(), L->n, src, L->ph.cf, L->stream);
    if (e) return hip_fail(e, "init kernel");
    if (!rho_on_device) {
        e = hipStreamSynchronize(L->stream);
        if (e) return hip_fail(e, "hipStreamSynchronize");
    }
    L->have_state = true;
    if (auto st = span_clear_error(L)) return st;
    L->step = 0;
    return KSLB_OK;
}

}  // extern "C"

namespace {

// Enqueue n_steps steps.  noalloc: the SPAN kernel's edge slots come from the
// library's static device area instead of the lattice's exchange area, and
// nothing is allocated.
kslb_status advance_impl(kslb_lattice* L, int64_t n_steps, bool noalloc)
{
    if (auto s = check_lat(L)) return s;
    if (n_steps < 0) return fail(KSLB_EINVAL, "n_steps must be >= 0");
    if (!L->have_state) return fail(KSLB_ESTATE, "advance before init_rho/write_f");
    if (n_steps == 0) return KSLB_OK;
    DeviceGuard g(L->device);
    const Limits lim = device_limits(L->q, L->prec, L->fixed);
    const KernelChoice kc = plan_kernel(L->n, L->q, L->prec, L->fixed, L->kernel, L->tile_steps, lim);
    const int kernel = kc.kernel;
    const int ringB = ring_sites_per_lane(L->n, L->q, lim.lds_bytes);
    if (L->fixed && kernel != KSLB_KERNEL_PLAIN && kernel != KSLB_KERNEL_SPAN)
        return fail(KSLB_EINVAL, "fixed ends run on the PLAIN and SPAN kernels only");
    int e = 0;
    if (kernel == KSLB_KERNEL_PLAIN && L->fixed) {
        for (int64_t s = 0; s < n_steps; s++) {
            e = launch_plain_fixed(L->q, L->prec, L->state(), L->other(), L->n, L->ph.cf, L->ends, L->stream);
            if (e) return hip_fail(e, "plain kernel");
            L->cur ^= 1;
        }
    } else if (kernel == KSLB_KERNEL_PLAIN) {
        for (int64_t s = 0; s < n_steps; s++) {
            e = launch_plain(L->q, L->prec, L->state(), L->other(), L->n, L->ph.cf, L->stream);
            if (e) return hip_fail(e, "plain kernel");
            L->cur ^= 1;
        }
    } else if (kernel == KSLB_KERNEL_SPAN) {
        const int sp = kc.steps;
        const int nwg = sp ? span_plan(L->n, L->q, L->prec, sp, lim.span_owners) : 0;
        if (!nwg)
            return fail(KSLB_EINVAL, "shape cannot use the multi-workgroup kernel (at most %lld resident workgroups)",
                        (long long)lim.span_owners);
        const int64_t ecopy = span_edge_copy_bytes(L->q, L->prec, L->n, nwg, sp);
        const int64_t per = (int64_t)nwg * ecopy;    // edge slots of one exchange
        int64_t slots = 0;
        char* ebase = nullptr;
        if (noalloc) {
            if ((size_t)per > kNoAllocScratchBytes)
                return fail(KSLB_ENOMEM, "one exchange of this lattice needs %lld bytes of edge slots; the static area "
                            "of the no-allocation advance holds %zu", (long long)per, kNoAllocScratchBytes);
            char* area = nullptr;
            if (int e2 = noalloc_scratch(&area)) return hip_fail(e2, "static exchange area");
            slots = span_slot_capacity(per, sp, kNoAllocScratchBytes);
            ebase = area;
        } else {
            if (auto st = span_prepare(L, per, sp, n_steps, &slots)) return st;
            ebase = L->span_scratch;
        }
        if (auto st = span_ctl_setup(L)) return st;
        int* ctl = L->ctl();
        // launches of equal length (to a multiple of sp), each within the slots
        const int64_t cap = std::min<int64_t>(kMaxStepsPerLaunch, (slots + 1) * sp);
        const int64_t nl = (n_steps + cap - 1) / cap;
        const int64_t chunk = std::min(cap, ((n_steps + nl - 1) / nl + sp - 1) / sp * sp);
        // failure-path testing: KSLB_SPAN_INJECT_ABORT=1 starts every launch
        // with its abort word raised
        const char* inj = std::getenv("KSLB_SPAN_INJECT_ABORT");
        const bool inject = inj && inj[0] == '1';
        for (int64_t done = 0; done < n_steps; done += chunk) {
            const int64_t s = std::min(chunk, n_steps - done);
            e = launch_span(L->q, L->prec, L->state(), L->other(), L->n, nwg, s, sp, ebase, ecopy, slots, ctl,
                            L->ph.cf, L->stream, L->fixed ? &L->ends : nullptr, inject);
            if (e) return hip_fail(e, "multi-workgroup kernel");
            L->cur ^= 1;
        }
    } else if (kernel == KSLB_KERNEL_RESIDENT) {
        if (!ringB) return fail(KSLB_EINVAL, "shape cannot use the resident kernel");
        const int64_t chunk = kMaxStepsPerLaunch;
        for (int64_t done = 0; done < n_steps; done += chunk) {
            const int64_t s = std::min(chunk, n_steps - done);
            e = launch_ring(L->q, L->prec, ringB, L->state(), L->other(), L->n, s, L->ph.cf, L->stream);
            if (e) return hip_fail(e, "resident kernel");
            L->cur ^= 1;
        }
    } else {
        const int s_max = kc.steps;
        for (int64_t done = 0; done < n_steps;) {
            const int s = (int)std::min<int64_t>(s_max, n_steps - done);
            e = launch_tile(L->q, L->prec, L->state(), L->other(), L->n, s, L->ph.cf,
                            L->stream);
            if (e) return hip_fail(e, "tiled kernel");
            L->cur ^= 1;
            done += s;
        }
    }
    L->step += n_steps;
    return KSLB_OK;
}

}  // namespace

extern "C" {

kslb_status kslb_advance(kslb_lattice* L, int64_t n_steps) { return advance_impl(L, n_steps, false); }

kslb_status kslb_solve(kslb_lattice* L, const double* rho0, int64_t n_steps, double* rho_out)
{
    if (auto s = check_lat(L)) return s;
    if (!rho0 || !rho_out) return fail(KSLB_EINVAL, "rho0 and rho_out must not be NULL");
    if (n_steps < 0) return fail(KSLB_EINVAL, "n_steps must be >= 0");
    if (!L->ph.set) return fail(KSLB_ESTATE, "set the coefficients before solve");
    DeviceGuard g(L->device);
    const Limits lim = device_limits(L->q, L->prec, L->fixed);
    const KernelChoice kc = plan_kernel(L->n, L->q, L->prec, L->fixed, L->kernel, L->tile_steps, lim);
    const bool aligned = reinterpret_cast<uintptr_t>(rho0) % 16 == 0 && reinterpret_cast<uintptr_t>(rho_out) % 16 == 0;
    if (kc.kernel != KSLB_KERNEL_TILED || L->fixed || n_steps == 0 || !aligned) {
        if (auto st = kslb_init_rho(L, rho0, 1)) return st;
        if (auto st = advance_impl(L, n_steps, false)) return st;
        return kslb_read_rho(L, rho_out, 1);
    }
    // tiled: the first launch forms the initial state from rho0 on load, the
    // last also writes the density; the state copies end as after the three
    // separate calls.  One launch that both reads rho0 and writes an
    // overlapping rho_out would race (a window stores its sites' densities
    // while a neighbouring window may still load them as halo), so then the
    // readout runs after it.
    const uintptr_t in0 = reinterpret_cast<uintptr_t>(rho0), out0 = reinterpret_cast<uintptr_t>(rho_out);
    const uintptr_t bytes = sizeof(double) * (uintptr_t)L->n;
    const bool overlap = out0 < in0 + bytes && in0 < out0 + bytes;
    const bool fuse_out = !(overlap && n_steps <= kc.steps);
    L->cur = 0;
    L->step = 0;
    if (auto st = span_clear_error(L)) return st;
    for (int64_t done = 0; done < n_steps;) {
        const int s = (int)std::min<int64_t>(kc.steps, n_steps - done);
        const bool first = done == 0, last = done + s == n_steps;
        int e = launch_tile(L->q, L->prec, L->state(), L->other(), L->n, s, L->ph.cf,
                            L->stream, first ? rho0 : nullptr, last && fuse_out ? rho_out : nullptr);
        if (e) {
            if (first) L->have_state = false;     // neither copy holds a state now
            return hip_fail(e, "tiled kernel");
        }
        L->have_state = true;
        L->cur ^= 1;
        done += s;
    }
    L->step = n_steps;
    return fuse_out ? KSLB_OK : kslb_read_rho(L, rho_out, 1);
}

kslb_status kslb_advance_noalloc(kslb_lattice* L, int64_t n_steps) { return advance_impl(L, n_steps, true); }

kslb_status kslb_read_rho(kslb_lattice* L, double* out, int out_on_device)
{
    if (auto s = check_lat(L)) return s;
    if (!out) return fail(KSLB_EINVAL, "out must not be NULL");
    if (!L->have_state) return fail(KSLB_ESTATE, "no state");
    DeviceGuard g(L->device);
    double* dst = out;
    if (!out_on_device) {
        if (auto s = ensure_staging(L)) return s;
        dst = L->staging;
    }
    int e = launch_read_rho(L->q, L->prec, L->state(), L->n, dst, L->stream, L->sticky());
    if (e) return hip_fail(e, "readout kernel");
    if (!out_on_device) {
        e = hipMemcpyAsync(out, dst, sizeof(double) * (size_t)L->n, hipMemcpyDeviceToHost, L->stream);
        if (e) return hip_fail(e, "hipMemcpyAsync(rho)");
        e = hipStreamSynchronize(L->stream);
        if (e) return hip_fail(e, "hipStreamSynchronize");
        return span_check_error(L);
    }
    return KSLB_OK;
}

kslb_status kslb_read_f(kslb_lattice* L, double* out, int out_on_device, int pre_collision)
{
    if (auto s = check_lat(L)) return s;
    if (!out) return fail(KSLB_EINVAL, "out must not be NULL");
    if (!L->have_state) return fail(KSLB_ESTATE, "no state");
    if (!L->ph.set) return fail(KSLB_ESTATE, "coefficients not set");
    DeviceGuard g(L->device);
    double* dst = out;
    if (!out_on_device) {
        if (auto s = ensure_staging(L)) return s;
        dst = L->staging;
    }
    int e = launch_read_f(L->q, L->prec, L->state(), L->n, dst, pre_collision ? 1 : 0, L->ph.cf, L->stream,
                          L->sticky());
    if (e) return hip_fail(e, "read_f kernel");
    if (!out_on_device) {
        e = hipMemcpyAsync(out, dst, sizeof(double) * (size_t)L->q * (size_t)L->n, hipMemcpyDeviceToHost,
                           L->stream);
        if (e) return hip_fail(e, "hipMemcpyAsync(f)");
        e = hipStreamSynchronize(L->stream);
        if (e) return hip_fail(e, "hipStreamSynchronize");
        return span_check_error(L);
    }
    return KSLB_OK;
}

kslb_status kslb_write_f(kslb_lattice* L, const double* in, int in_on_device, int64_t step)
{
    if (auto s = check_lat(L)) return s;
    if (!in) return fail(KSLB_EINVAL, "in must not be NULL");
    if (!L->ph.set) return fail(KSLB_ESTATE, "coefficients not set");
    if (step < 0) return fail(KSLB_EINVAL, "step must be >= 0");
    DeviceGuard g(L->device);
    const double* src = in;
    if (!in_on_device) {
        if (auto s = ensure_staging(L)) return s;
        int e = hipMemcpyAsync(L->staging, in, sizeof(double) * (size_t)L->q * (size_t)L->n,
                               hipMemcpyHostToDevice, L->stream);
        if (e) return hip_fail(e, "hipMemcpyAsync(f)");
        src = L->staging;
    }
    L->cur = 0;
    int e = launch_write_f(L->q, L->prec, L->state(), L->n, src, L->ph.cf, L->stream);
    if (e) return hip_fail(e, "write_f kernel");
    if (!in_on_device) {
        e = hipStreamSynchronize(L->stream);
        if (e) return hip_fail(e, "hipStreamSynchronize");
    }
    L->have_state = true;
    if (auto st = span_clear_error(L)) return st;
    L->step = step;
    return KSLB_OK;
}

size_t kslb_state_size(const kslb_lattice* L) { return L ? L->copy : 0; }

kslb_status kslb_save_state(kslb_lattice* L, void* dev_dst)
{
    if (auto s = check_lat(L)) return s;
    if (!dev_dst) return fail(KSLB_EINVAL, "null destination");
    if (!L->have_state) return fail(KSLB_ESTATE, "no state");
    DeviceGuard g(L->device);
    // a checkpoint of a state a multi-workgroup launch left invalid is refused
    if (auto st = span_check_error(L)) return st;
    int e = hipMemcpyAsync(dev_dst, L->state(), L->copy, hipMemcpyDeviceToDevice, L->stream);
    if (e) return hip_fail(e, "hipMemcpyAsync(save)");
    return KSLB_OK;
}

kslb_status kslb_load_state(kslb_lattice* L, const void* dev_src, int64_t step)
{
    if (auto s = check_lat(L)) return s;
    if (!dev_src) return fail(KSLB_EINVAL, "null source");
    if (step < 0) return fail(KSLB_EINVAL, "step must be >= 0");
    DeviceGuard g(L->device);
    L->cur = 0;
    int e = hipMemcpyAsync(L->state(), dev_src, L->copy, hipMemcpyDeviceToDevice, L->stream);
    if (e) return hip_fail(e, "hipMemcpyAsync(load)");
    L->have_state = true;
    if (auto st = span_clear_error(L)) return st;
    L->step = step;
    return KSLB_OK;
}

kslb_status kslb_step_count(const kslb_lattice* L, int64_t* step)
{
    if (auto s = check_lat(L)) return s;
    if (!step) return fail(KSLB_EINVAL, "step must not be NULL");
    *step = L->step;
    return KSLB_OK;
}

kslb_status kslb_diagnostics(kslb_lattice* L, double* mass, int* nonfinite)
{
    if (auto s = check_lat(L)) return s;
    if (!L->have_state) return fail(KSLB_ESTATE, "no state");
    DeviceGuard g(L->device);
    double* partial = L->diag();
    double* mass_d = partial + 256;
    int* flag_d = reinterpret_cast<int*>(partial + 257);
    int e = launch_diag(L->q, L->prec, L->state(), L->n, partial, flag_d, mass_d, L->stream);
    if (e) return hip_fail(e, "diagnostics kernel");
    double m = 0.0;
    int f = 0;
    e = hipMemcpyAsync(&m, mass_d, sizeof m, hipMemcpyDeviceToHost, L->stream);
    if (!e) e = hipMemcpyAsync(&f, flag_d, sizeof f, hipMemcpyDeviceToHost, L->stream);
    if (!e) e = hipStreamSynchronize(L->stream);
    if (e) return hip_fail(e, "diagnostics copy");
    if (mass) *mass = m;
    if (nonfinite) *nonfinite = f;
    return span_check_error(L);
}

kslb_status kslb_aborted_launches(kslb_lattice* L, int64_t* count)
{
    if (auto s = check_lat(L)) return s;
    if (!count) return fail(KSLB_EINVAL, "count must not be NULL");
    *count = 0;
    if (!L->ctl_ready) return KSLB_OK;
    DeviceGuard g(L->device);
    int c = 0;
    int e = hipMemcpyAsync(&c, L->ctl() + span_ctl_aborts_index(), sizeof c, hipMemcpyDeviceToHost, L->stream);
    if (!e) e = hipStreamSynchronize(L->stream);
    if (e) return hip_fail(e, "SPAN control copy");
    *count = c;
    return KSLB_OK;
}

kslb_status kslb_destroy(kslb_lattice* L)
{
    if (!L) return KSLB_OK;
    if (L->staging || L->span_scratch) {
        DeviceGuard g(L->device);
        (void)hipStreamSynchronize(L->stream);
        if (L->staging) (void)hipFree(L->staging);
        if (L->span_scratch) (void)hipFree(L->span_scratch);
    }
    delete L;
    return KSLB_OK;
}

const char* kslb_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ============================================================================
// ensemble
// ============================================================================

struct kslb_ensemble {
    int count = 0, device = 0;
    char* buf = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    std::vector<int> q, prec;          // scheme and storage of each instance
    std::vector<int64_t> cap, n;       // capacity and current size (sites) per instance
    // device address of copy 0 (in buf, or in caller memory for an instance
    // bound elsewhere) and bytes per copy (at capacity)
    std::vector<uintptr_t> addr;
    std::vector<size_t> copy;
    uint64_t layout_gen = 1;           // changes whenever an instance is bound to other memory
    std::vector<int> cur;
    std::vector<int64_t> step;
    std::vector<char> have_state;
    // Coefficient sets: instance i uses set cls[i] (-1: not set yet), of
    // scheme set_q[k].  gen changes whenever any instance's set changes.
    std::vector<int> cls;
    std::vector<Physics> sets;
    std::vector<int> set_q;
    uint64_t coef_gen = 1;
    // defaults: the fastest of the tuner's grid for the 4096-instance workload
    // (64-step chunks: 783 GLUPS against 739 for 32)
    int B = 8, chunk = 64, max_seg = 16;
    size_t diag_off = 0;
    // Descriptor tables (window headers, segments, coefficient sets): two
    // device slots (one per ping-pong parity), each remembered by the
    // signature of the plan it holds, with the launches of that plan.
    struct Launch { int q, prec, w0, nwin; };
    char* d_tab[2] = {nullptr, nullptr};
    size_t d_cap[2] = {0, 0};
    std::vector<uint64_t> sig[2];
    std::vector<Launch> launches[2];
    size_t seg_at[2] = {0, 0}, coef_at[2] = {0, 0};   // byte offsets in the slot
    int next_slot = 0;
    char* h_pin[2] = {nullptr, nullptr};   // pinned staging of each slot's upload
    size_t h_cap[2] = {0, 0};
    hipEvent_t up_ev[2] = {nullptr, nullptr};
    bool up_pending[2] = {false, false};
    uint64_t slot_gen[2] = {0, 0};          // bumped whenever a slot is rewritten
    // steady state: the two alternating chunks' launches captured as one graph
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;       // private stream the graph is recorded on
    hipGraphExec_t gexec = nullptr;
    uint64_t gkey[5] = {0, 0, 0, 0, 0};
    uint64_t gseen[5] = {0, 0, 0, 0, 0};    // last pair of plans that ran eagerly
    std::vector<std::pair<hipGraphExec_t, hipEvent_t>> retired;   // graphs that may still run
    double* staging = nullptr;
    int64_t staging_n = 0;
    // batched init and readout: descriptor (and coefficient) tables, each
    // with its pinned staging and the event of its last upload
    struct Table {
        char* d = nullptr;
        char* h = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    Table init_tab, read_tab, group_tab;
    // trajectory pairs: device table and its pinned staging
    char* d_pairs = nullptr;
    char* h_pairs = nullptr;
    size_t pairs_cap = 0;
    hipEvent_t pairs_ev = nullptr;
    bool pairs_pending = false;
};

namespace {

// Byte offsets of the instances' copy 0 in an ensemble buffer and bytes per
// copy; returns the bytes of all instances' states.
size_t ens_layout(int count, const int64_t* n_sites, const int* q, const int* prec, std::vector<size_t>* off,
                  std::vector<size_t>* copy)
{
    size_t pos = 0;
    for (int i = 0; i < count; i++) {
        const size_t c = state_copy_bytes(n_sites[i], q[i], prec[i]);
        if (off) off->push_back(pos);
        if (copy) copy->push_back(c);
        pos += 2 * c;
    }
    return pos;
}

kslb_status check_ens(const kslb_ensemble* E, int idx)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    if (idx < 0 || idx >= E->count) return fail(KSLB_EINVAL, "instance %d out of range [0, %d)", idx, E->count);
    return KSLB_OK;
}

kslb_status ens_staging(kslb_ensemble* E, int64_t n)
{
    if (E->staging && E->staging_n >= n) return KSLB_OK;
    if (E->staging) {
        (void)hipStreamSynchronize(E->stream);
        (void)hipFree(E->staging);
        E->staging = nullptr;
    }
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(double) * (size_t)n)) return fail(KSLB_ENOMEM, "staging allocation failed");
    E->staging = (double*)p;
    E->staging_n = n;
    return KSLB_OK;
}

// Device address of copy `which` (0 or 1) of instance i.
uint64_t ens_addr(const kslb_ensemble* E, int i, int which)
{
    return (uint64_t)(E->addr[i] + (uintptr_t)which * E->copy[i]);
}

char* ens_state(kslb_ensemble* E, int i) { return reinterpret_cast<char*>(ens_addr(E, i, E->cur[i])); }

int ens_max_halo(const kslb_ensemble* E)
{
    int h = 0;
    for (int i = 0; i < E->count; i++) h = std::max(h, halo(E->q[i]));
    return h;
}

// Give instance i (every instance for i < 0) the coefficient set ph of
// scheme q, sharing an equal set already held.  Sets no instance uses are
// dropped once they outnumber the instances.
void ens_assign(kslb_ensemble* E, int i, int q, const Physics& ph)
{
    int k = -1;
    for (size_t j = 0; j < E->sets.size(); j++)
        if (E->set_q[j] == q && E->sets[j].tau == ph.tau && std::memcmp(&E->sets[j].cf, &ph.cf, sizeof(Coef)) == 0) {
            k = (int)j;
            break;
        }
    if (k < 0) {
        E->sets.push_back(ph);
        E->set_q.push_back(q);
        k = (int)E->sets.size() - 1;
    }
    for (int j = 0; j < E->count; j++)
        if (j == i || (i < 0 && E->q[j] == q)) E->cls[j] = k;
    E->coef_gen++;
    if ((int)E->sets.size() > E->count + 8) {
        std::vector<int> map(E->sets.size(), -1);
        std::vector<Physics> sets;
        std::vector<int> set_q;
        for (int j = 0; j < E->count; j++) {
            const int c = E->cls[j];
            if (c < 0) continue;
            if (map[c] < 0) {
                map[c] = (int)sets.size();
                sets.push_back(E->sets[c]);
                set_q.push_back(E->set_q[c]);
            }
            E->cls[j] = map[c];
        }
        E->sets.swap(sets);
        E->set_q.swap(set_q);
    }
}

struct Tile {
    int inst;
    int64_t start;
    int32_t valid;
    int lanes;
};

// A planned chunk: the launches (one per scheme and storage present), their
// windows in the slot's header table, and the slot's segment and coefficient
// tables.
struct EnsPlan {
    const WinHdr* hdr = nullptr;
    const SegDesc* seg = nullptr;
    const Coef* coefs = nullptr;
    const std::vector<kslb_ensemble::Launch>* launches = nullptr;
    int slot = 0;
    int nwin = 0;
};

void ens_plan_view(const kslb_ensemble* E, int k, EnsPlan* plan)
{
    plan->hdr = reinterpret_cast<const WinHdr*>(E->d_tab[k]);
    plan->seg = reinterpret_cast<const SegDesc*>(E->d_tab[k] + E->seg_at[k]);
    plan->coefs = reinterpret_cast<const Coef*>(E->d_tab[k] + E->coef_at[k]);
    plan->launches = &E->launches[k];
    plan->slot = k;
    plan->nwin = 0;
    for (const auto& l : E->launches[k]) plan->nwin += l.nwin;
}

// Build and upload the descriptor tables of one chunk (instances advancing
// s_i = adv[i] > 0 steps), or reuse a device slot that already holds the same
// plan.  Tiles of at most W - 2 H s sites (a multiple of B) cut each
// instance; best-fit-decreasing packs tiles of one scheme, storage, step
// count and coefficient set into windows of tile_lanes() lanes and at most
// max_seg segments.  Windows are ordered by scheme and storage, one launch
// each.
kslb_status ens_plan(kslb_ensemble* E, const std::vector<int>& adv, EnsPlan* plan, int avoid = -1)
{
    std::vector<uint64_t> key;
    key.reserve(3 * (size_t)E->count + 4);
    key.push_back((uint64_t)E->B);
    key.push_back((uint64_t)E->max_seg);
    key.push_back(E->coef_gen);
    key.push_back(E->layout_gen);
    for (int i = 0; i < E->count; i++) {
        if (adv[i] <= 0) continue;
        key.push_back((uint64_t)i);
        key.push_back(((uint64_t)adv[i] << 1) | (uint64_t)E->cur[i]);
        key.push_back((uint64_t)E->n[i]);
    }
    for (int k = 0; k < 2; k++) {
        if (E->d_tab[k] && E->sig[k] == key) {
            ens_plan_view(E, k, plan);
            return KSLB_OK;
        }
    }
    const int B = E->B;
    const int LANES = tile_lanes();
    const int64_t W = (int64_t)LANES * B;
    // a tile's packing class: scheme, storage, steps, coefficient set
    struct Cls {
        int q, prec, steps, coef;
        bool operator==(const Cls& o) const
        {
            return q == o.q && prec == o.prec && steps == o.steps && coef == o.coef;
        }
    };
    std::vector<std::pair<Cls, Tile>> tiles;
    for (int i = 0; i < E->count; i++) {
        const int st = adv[i];
        if (st <= 0) continue;
        const int64_t hs = (int64_t)halo(E->q[i]) * st;
        int64_t tmax = W - 2 * hs;
        tmax -= tmax % B;
        const int64_t n = E->n[i];
        for (int64_t t0 = 0; t0 < n; t0 += tmax) {
            Tile t;
            t.inst = i;
            t.start = t0 - hs;
            t.valid = (int32_t)std::min<int64_t>(tmax, n - t0);
            t.lanes = (int)((t.valid + 2 * hs + B - 1) / B);
            tiles.push_back({Cls{E->q[i], E->prec[i], st, E->cls[i]}, t});
        }
    }
    std::sort(tiles.begin(), tiles.end(), [](const std::pair<Cls, Tile>& a, const std::pair<Cls, Tile>& b) {
        const Cls &x = a.first, &y = b.first;
        if (x.q != y.q) return x.q < y.q;
        if (x.prec != y.prec) return x.prec < y.prec;
        if (x.steps != y.steps) return x.steps > y.steps;
        if (x.coef != y.coef) return x.coef < y.coef;
        return a.second.lanes > b.second.lanes;
    });
    struct Win { Cls c; int used; std::vector<Tile> t; };
    std::vector<Win> wins;
    size_t g0 = 0;
    while (g0 < tiles.size()) {
        const Cls c = tiles[g0].first;
        size_t g1 = g0;
        while (g1 < tiles.size() && tiles[g1].first == c) g1++;
        std::multimap<int, size_t> free_lanes;   // remaining lanes -> window index
        for (size_t k = g0; k < g1; k++) {
            const Tile& t = tiles[k].second;
            auto it = free_lanes.lower_bound(t.lanes);
            size_t w;
            if (it == free_lanes.end()) {
                wins.push_back(Win{c, 0, {}});
                w = wins.size() - 1;
            } else {
                w = it->second;
                free_lanes.erase(it);
            }
            wins[w].t.push_back(t);
            wins[w].used += t.lanes;
            const int left = LANES - wins[w].used;
            if (left >= B && (int)wins[w].t.size() < E->max_seg) free_lanes.insert({left, w});
        }
        g0 = g1;
    }
    std::vector<WinHdr> hv;
    std::vector<SegDesc> sv;
    std::vector<kslb_ensemble::Launch> lv;
    hv.reserve(wins.size());
    for (const Win& w : wins) {
        if (lv.empty() || lv.back().q != w.c.q || lv.back().prec != w.c.prec)
            lv.push_back(kslb_ensemble::Launch{w.c.q, w.c.prec, (int)hv.size(), 0});
        lv.back().nwin++;
        WinHdr h;
        h.first_seg = (int32_t)sv.size();
        h.nseg = (int32_t)w.t.size();
        h.steps = w.c.steps;
        h.coef = w.c.coef;
        hv.push_back(h);
        int lane = 0;
        for (const Tile& t : w.t) {
            const int i = t.inst;
            SegDesc d;
            d.src = ens_addr(E, i, E->cur[i]);
            d.dst = ens_addr(E, i, 1 - E->cur[i]);
            d.n = E->n[i];
            d.pitch = state_pitch(E->n[i]);
            d.start = t.start;
            d.lane_lo = lane;
            d.valid = t.valid;
            sv.push_back(d);
            lane += t.lanes;
        }
    }
    const size_t seg_at = sizeof(WinHdr) * hv.size();
    const size_t coef_at = seg_at + sizeof(SegDesc) * sv.size();
    const size_t bytes = coef_at + sizeof(Coef) * E->sets.size();
    int k = E->next_slot;
    if (k == avoid) k ^= 1;
    E->next_slot = k ^ 1;
    E->slot_gen[k]++;
    E->sig[k].clear();   // the slot holds no valid plan until the upload below is enqueued
    // the tables grow geometrically: an ensemble whose active set grows call
    // by call (continuous admission) reallocates, and waits for its stream,
    // a logarithmic number of times
    if (E->d_cap[k] < bytes) {
        const size_t want = std::max(bytes, 2 * E->d_cap[k]);
        if (E->d_tab[k]) {
            (void)hipStreamSynchronize(E->stream);
            (void)hipFree(E->d_tab[k]);
            E->d_tab[k] = nullptr;
            E->d_cap[k] = 0;
        }
        void* p = nullptr;
        if (hipMalloc(&p, want)) return fail(KSLB_ENOMEM, "descriptor allocation of %zu bytes failed", want);
        E->d_tab[k] = (char*)p;
        E->d_cap[k] = want;
    }
    // pinned staging: wait for this slot's previous upload before rewriting it
    if (E->up_pending[k]) {
        int e = hipEventSynchronize(E->up_ev[k]);
        if (e) return hip_fail(e, "hipEventSynchronize");
        E->up_pending[k] = false;
    }
    if (E->h_cap[k] < bytes) {
        const size_t want = std::max(bytes, 2 * E->h_cap[k]);
        if (E->h_pin[k]) (void)hipHostFree(E->h_pin[k]);
        E->h_pin[k] = nullptr;
        E->h_cap[k] = 0;
        void* hp = nullptr;
        if (hipHostMalloc(&hp, want, hipHostMallocDefault)) return fail(KSLB_ENOMEM, "pinned staging allocation failed");
        E->h_pin[k] = (char*)hp;
        E->h_cap[k] = want;
    }
    if (!E->up_ev[k] && hipEventCreateWithFlags(&E->up_ev[k], hipEventDisableTiming))
        return fail(KSLB_EDEVICE, "hipEventCreate failed");
    std::memcpy(E->h_pin[k], hv.data(), seg_at);
    std::memcpy(E->h_pin[k] + seg_at, sv.data(), coef_at - seg_at);
    for (size_t j = 0; j < E->sets.size(); j++)
        std::memcpy(E->h_pin[k] + coef_at + j * sizeof(Coef), &E->sets[j].cf, sizeof(Coef));
    // stream order keeps earlier kernels reading this slot ahead of the copy
    int e = hipMemcpyAsync(E->d_tab[k], E->h_pin[k], bytes, hipMemcpyHostToDevice, E->stream);
    if (!e) e = hipEventRecord(E->up_ev[k], E->stream);
    if (e) return hip_fail(e, "descriptor upload");
    E->up_pending[k] = true;
    E->sig[k] = key;
    E->launches[k] = lv;
    E->seg_at[k] = seg_at;
    E->coef_at[k] = coef_at;
    ens_plan_view(E, k, plan);
    return KSLB_OK;
}

// Enqueue a planned chunk: one kernel per scheme and storage present.
int ens_launch(const kslb_ensemble* E, const EnsPlan& plan, hipStream_t stream)
{
    for (const auto& l : *plan.launches) {
        int e = launch_ens(l.q, l.prec, E->B, plan.hdr + l.w0, plan.seg, l.nwin, plan.coefs, stream);
        if (e) return e;
    }
    return 0;
}

// Replays of one pair of plans within a call from which recording a graph pays.
constexpr int64_t kGraphMinPairs = 4;

// Retire the current graph: record an event behind its replays on the
// ensemble's stream and keep both until the event has completed.
kslb_status ens_retire_graph(kslb_ensemble* E)
{
    hipEvent_t ev = nullptr;
    int e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (!e) e = hipEventRecord(ev, E->stream);
    if (e) {
        if (ev) (void)hipEventDestroy(ev);
        return hip_fail(e, "graph retirement event");
    }
    E->retired.push_back({E->gexec, ev});
    E->gexec = nullptr;
    return KSLB_OK;
}

// Destroy the retired graphs whose replays have completed (all of them,
// waiting, when wait is set).
void ens_reap_graphs(kslb_ensemble* E, bool wait)
{
    size_t keep = 0;
    for (size_t k = 0; k < E->retired.size(); k++) {
        auto& r = E->retired[k];
        const bool done = wait ? hipEventSynchronize(r.second) == hipSuccess : hipEventQuery(r.second) == hipSuccess;
        if (done || wait) {
            (void)hipGraphExecDestroy(r.first);
            (void)hipEventDestroy(r.second);
        } else {
            E->retired[keep++] = r;
        }
    }
    E->retired.resize(keep);
}

// Steady state: every active instance has at least `pairs` * 2 more full
// chunks.  The chunk with the current parities and the one after it (all
// parities flipped) are planned into the two descriptor slots and captured
// as a graph of their kernel launches, replayed `pairs` times (or launched
// directly, see below).  The graph holds kernels only (no memset or copy
// nodes); it is rebuilt whenever either slot is rewritten.
kslb_status ens_replay_pairs(kslb_ensemble* E, const std::vector<int>& adv, int64_t pairs)
{
    EnsPlan pa, pb;
    if (auto s = ens_plan(E, adv, &pa)) return s;
    for (int i = 0; i < E->count; i++)
        if (adv[i] > 0) E->cur[i] ^= 1;
    kslb_status st = ens_plan(E, adv, &pb, pa.slot);
    for (int i = 0; i < E->count; i++)
        if (adv[i] > 0) E->cur[i] ^= 1;
    if (st) return st;
    const uint64_t key[5] = {(uint64_t)pa.slot, E->slot_gen[pa.slot], (uint64_t)pb.slot, E->slot_gen[pb.slot],
                             ((uint64_t)E->B << 32) | (uint64_t)(pa.nwin + pb.nwin)};
    if (!E->gexec || std::memcmp(key, E->gkey, sizeof key) != 0) {
        // Recording and instantiating a graph pays for a pair of plans that
        // one call replays at least kGraphMinPairs times or that recurs; a
        // layout that changes every call (continuous admission) launches
        // directly.
        if (pairs < kGraphMinPairs && std::memcmp(key, E->gseen, sizeof key) != 0) {
            std::memcpy(E->gseen, key, sizeof key);
            for (int64_t r = 0; r < pairs; r++) {
                int e = ens_launch(E, pa, E->stream);
                if (!e) e = ens_launch(E, pb, E->stream);
                if (e) return hip_fail(e, "ensemble kernel");
            }
            return KSLB_OK;
        }
        // the previous graph may still run: it is destroyed once an event
        // recorded after its last replay has completed, without waiting here
        if (E->gexec) {
            if (auto st = ens_retire_graph(E)) return st;
        }
        ens_reap_graphs(E, false);
        // record on a private stream (the caller's may be the null stream,
        // which cannot be captured); replay on the caller's stream
        if (!E->cap_stream) {
            int e = hipStreamCreateWithFlags(&E->cap_stream, hipStreamNonBlocking);
            if (e) return hip_fail(e, "hipStreamCreateWithFlags");
        }
        hipGraph_t graph = nullptr;
        int e = hipStreamBeginCapture(E->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e) return hip_fail(e, "hipStreamBeginCapture");
        int e1 = ens_launch(E, pa, E->cap_stream);
        int e2 = e1 ? 0 : ens_launch(E, pb, E->cap_stream);
        e = hipStreamEndCapture(E->cap_stream, &graph);
        if (e1 || e2 || e) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(e1 ? e1 : (e2 ? e2 : e), "ensemble graph capture");
        }
        e = hipGraphInstantiate(&E->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e) {
            E->gexec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        std::memcpy(E->gkey, key, sizeof key);
    }
    for (int64_t r = 0; r < pairs; r++) {
        int e = hipGraphLaunch(E->gexec, E->stream);
        if (e) return hip_fail(e, "hipGraphLaunch");
    }
    return KSLB_OK;
}

// Stage `bytes` of host data into table t and enqueue its upload on the
// ensemble's stream; *dev receives the device copy.  The pinned staging is
// rewritten only after its previous upload has completed.
kslb_status ens_upload(kslb_ensemble* E, kslb_ensemble::Table& t, const void* data, size_t bytes, char** dev)
{
    int e = 0;
    if (t.pending) {
        e = hipEventSynchronize(t.ev);
        if (e) return hip_fail(e, "table upload event");
        t.pending = false;
    }
    if (t.cap < bytes) {
        if (t.d) {
            (void)hipStreamSynchronize(E->stream);
            (void)hipFree(t.d);
        }
        if (t.h) (void)hipHostFree(t.h);
        t.d = t.h = nullptr;
        t.cap = 0;
        void* dp = nullptr;
        void* hp = nullptr;
        if (hipMalloc(&dp, bytes)) return fail(KSLB_ENOMEM, "table of %zu bytes", bytes);
        if (hipHostMalloc(&hp, bytes, hipHostMallocDefault)) {
            (void)hipFree(dp);
            return fail(KSLB_ENOMEM, "pinned table of %zu bytes", bytes);
        }
        t.d = (char*)dp;
        t.h = (char*)hp;
        t.cap = bytes;
    }
    if (!t.ev && hipEventCreateWithFlags(&t.ev, hipEventDisableTiming))
        return fail(KSLB_EDEVICE, "event creation failed");
    std::memcpy(t.h, data, bytes);
    e = hipMemcpyAsync(t.d, t.h, bytes, hipMemcpyHostToDevice, E->stream);
    if (!e) e = hipEventRecord(t.ev, E->stream);
    if (e) return hip_fail(e, "table upload");
    t.pending = true;
    *dev = t.d;
    return KSLB_OK;
}

void ens_table_free(kslb_ensemble::Table& t)
{
    if (t.d) (void)hipFree(t.d);
    if (t.h) (void)hipHostFree(t.h);
    if (t.ev) (void)hipEventDestroy(t.ev);
    t = kslb_ensemble::Table{};
}

// One launch's share of a batched init or readout: table rows [begin, end),
// all of one scheme and storage, sizes up to max_n.
struct InstGroup {
    int begin, end, q, prec;
    int64_t max_n;
};

// Instances in (scheme, storage) order with their packed-density offsets
// (instance order) and the state copy copy_of(i); *groups receives the runs.
template <class CopyOf>
std::vector<InstDesc> ens_inst_table(const kslb_ensemble* E, CopyOf copy_of, int64_t* total,
                                     std::vector<InstGroup>* groups)
{
    std::vector<int> order(E->count);
    for (int i = 0; i < E->count; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return E->q[a] != E->q[b] ? E->q[a] < E->q[b] : E->prec[a] < E->prec[b];
    });
    std::vector<int64_t> rho_off((size_t)E->count);
    int64_t pos = 0;
    for (int i = 0; i < E->count; i++) {
        rho_off[i] = pos;
        pos += E->n[i];
    }
    *total = pos;
    std::vector<InstDesc> dv((size_t)E->count);
    groups->clear();
    for (int k = 0; k < E->count; k++) {
        const int i = order[k];
        dv[k] = InstDesc{ens_addr(E, i, copy_of(i)), rho_off[i], E->n[i],
                         state_pitch(E->n[i]), std::max(E->cls[i], 0), 0};
        if (groups->empty() || groups->back().q != E->q[i] || groups->back().prec != E->prec[i])
            groups->push_back(InstGroup{k, k, E->q[i], E->prec[i], 0});
        groups->back().end = k + 1;
        groups->back().max_n = std::max(groups->back().max_n, E->n[i]);
    }
    return dv;
}

}  // namespace

extern "C" {

size_t kslb_ensemble_bytes(int count, const int64_t* n_sites, const int* q, const int* precision)
{
    if (count <= 0 || !n_sites || !q || !precision) return 0;
    for (int i = 0; i < count; i++)
        if (!valid_shape(n_sites[i], q[i], precision[i])) return 0;
    return ens_layout(count, n_sites, q, precision, nullptr, nullptr) + kDiagBytes;
}

kslb_status kslb_ensemble_create(kslb_ensemble** out, int count, const int64_t* n_sites, const int* q,
                                 const int* precision, void* dev_buf, size_t buf_bytes, void* hip_stream)
{
    if (!out) return fail(KSLB_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (count <= 0 || !n_sites || !q || !precision) return fail(KSLB_EINVAL, "count must be > 0 with sizes, schemes and storage modes");
    for (int i = 0; i < count; i++)
        if (!valid_shape(n_sites[i], q[i], precision[i]))
            return fail(KSLB_EINVAL, "bad shape of instance %d", i);
    if (!dev_buf || reinterpret_cast<uintptr_t>(dev_buf) % 256)
        return fail(KSLB_EINVAL, "device buffer missing or not 256-byte aligned");
    const size_t need = kslb_ensemble_bytes(count, n_sites, q, precision);
    if (buf_bytes < need) return fail(KSLB_ENOMEM, "buffer has %zu bytes, needs %zu", buf_bytes, need);
    int dev = 0;
    int e = hipGetDevice(&dev);
    if (e) return hip_fail(e, "hipGetDevice");
    kslb_ensemble* E = new (std::nothrow) kslb_ensemble;
    if (!E) return fail(KSLB_ENOMEM, "host allocation failed");
    E->count = count;
    E->q.assign(q, q + count);
    E->prec.assign(precision, precision + count);
    // FP64 throughout: 12 sites per lane by default (3072-site windows: 862
    // against 796 GLUPS for 4096 D1Q7 instances of 512 to 8192 sites); FP32
    // throughout: 10 sites and 48-step chunks (826-830 GLUPS, 783 at 64;
    // 799 at 8 sites); split storage present: 40-step chunks (485, 456 at 64)
    if (std::all_of(precision, precision + count, [](int p) { return p == kFP64; })) E->B = 12;
    if (std::all_of(precision, precision + count, [](int p) { return p == kFP32; })) {
        E->B = 10;
        E->chunk = 48;
    }
    if (std::any_of(precision, precision + count, [](int p) { return p == kSPLIT; })) E->chunk = 40;
    E->device = dev;
    E->buf = (char*)dev_buf;
    E->bytes = buf_bytes;
    E->stream = (hipStream_t)hip_stream;
    E->cap.assign(n_sites, n_sites + count);
    E->n = E->cap;
    std::vector<size_t> off;
    E->diag_off = ens_layout(count, n_sites, q, precision, &off, &E->copy);
    E->addr.resize(count);
    for (int i = 0; i < count; i++) E->addr[i] = reinterpret_cast<uintptr_t>(E->buf) + off[i];
    E->cur.assign(count, 0);
    E->step.assign(count, 0);
    E->have_state.assign(count, 0);
    E->cls.assign(count, -1);
    *out = E;
    return KSLB_OK;
}

kslb_status kslb_ensemble_set_physical(kslb_ensemble* E, int idx, double dX, double dT, double tau, int dm_variant,
                                       int guard_policy, double rho_max)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    if (idx >= 0) {
        if (auto s = check_ens(E, idx)) return s;
        Physics ph;
        kslb_status st = set_physics(ph, E->q[idx], dX, dT, tau, dm_variant, guard_policy, rho_max);
        if (st) return st;
        if ((st = rho_mode_check(E->prec[idx], ph))) return st;
        ens_assign(E, idx, E->q[idx], ph);
        return KSLB_OK;
    }
    // every instance: one set per scheme present, all checked before any is assigned
    Physics ph[2];
    bool want[2] = {false, false};
    for (int i = 0; i < E->count; i++) want[E->q[i] == 7] = true;
    for (int s = 0; s < 2; s++) {
        if (!want[s]) continue;
        kslb_status st = set_physics(ph[s], s ? 7 : 5, dX, dT, tau, dm_variant, guard_policy, rho_max);
        if (st) return st;
    }
    for (int i = 0; i < E->count; i++)
        if (auto st = rho_mode_check(E->prec[i], ph[E->q[i] == 7])) return st;
    for (int s = 0; s < 2; s++)
        if (want[s]) ens_assign(E, -1, s ? 7 : 5, ph[s]);
    return KSLB_OK;
}

kslb_status kslb_ensemble_get_tau(const kslb_ensemble* E, int idx, double* tau)
{
    if (auto s = check_ens(E, idx)) return s;
    if (!tau) return fail(KSLB_EINVAL, "tau must not be NULL");
    if (E->cls[idx] < 0) return fail(KSLB_ESTATE, "coefficients of instance %d not set", idx);
    *tau = E->sets[E->cls[idx]].tau;
    return KSLB_OK;
}

kslb_status kslb_ensemble_set_tiling(kslb_ensemble* E, int sites_per_lane, int max_segments, int steps_per_chunk)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    int B = sites_per_lane ? sites_per_lane : E->B;
    int m = max_segments ? max_segments : E->max_seg;
    int c = steps_per_chunk ? steps_per_chunk : E->chunk;
    bool all_rho = true, all_fp64 = true, all_fp32 = true;
    for (int i = 0; i < E->count; i++) {
        all_rho = all_rho && E->prec[i] == kRHO;
        all_fp64 = all_fp64 && E->prec[i] == kFP64;
        all_fp32 = all_fp32 && E->prec[i] == kFP32;
    }
    if (B != 4 && B != 8 && !(B == 10 && all_fp32) && !(B == 12 && all_fp64) && !(B == 16 && all_rho))
        return fail(KSLB_EINVAL, "sites_per_lane must be 4 or 8 (10 with FP32 storage throughout, 12 with FP64 "
                                 "storage throughout, 16 with the rho-only storage throughout)");
    if (m < 1 || m > tile_lanes()) return fail(KSLB_EINVAL, "max_segments must lie in [1, %d]", tile_lanes());
    const int64_t W = (int64_t)tile_lanes() * B;
    if (c < 1 || W - 2 * ens_max_halo(E) * (int64_t)c < B)
        return fail(KSLB_EINVAL, "steps_per_chunk %d leaves no valid sites in a %lld-site window", c, (long long)W);
    E->B = B;
    E->max_seg = m;
    E->chunk = c;
    return KSLB_OK;
}

kslb_status kslb_ensemble_get_tiling(const kslb_ensemble* E, int* sites_per_lane, int* max_segments,
                                     int* steps_per_chunk)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    if (sites_per_lane) *sites_per_lane = E->B;
    if (max_segments) *max_segments = E->max_seg;
    if (steps_per_chunk) *steps_per_chunk = E->chunk;
    return KSLB_OK;
}

kslb_status kslb_ensemble_set_graphs(kslb_ensemble* E, int enable)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    E->use_graphs = enable != 0;
    return KSLB_OK;
}

kslb_status kslb_ensemble_resize(kslb_ensemble* E, int idx, int64_t n_sites)
{
    if (auto s = check_ens(E, idx)) return s;
    if (n_sites <= 0 || n_sites > E->cap[idx])
        return fail(KSLB_EINVAL, "size %lld exceeds the capacity %lld of instance %d", (long long)n_sites,
                    (long long)E->cap[idx], idx);
    E->n[idx] = n_sites;
    E->have_state[idx] = 0;
    E->step[idx] = 0;
    return KSLB_OK;
}

size_t kslb_instance_bytes(int64_t n_sites, int q, int precision)
{
    if (!valid_shape(n_sites, q, precision)) return 0;
    return 2 * state_copy_bytes(n_sites, q, precision);
}

kslb_status kslb_ensemble_bind(kslb_ensemble* E, int idx, int64_t n_sites, void* dev_state, size_t bytes)
{
    if (auto s = check_ens(E, idx)) return s;
    if (!valid_shape(n_sites, E->q[idx], E->prec[idx]))
        return fail(KSLB_EINVAL, "bad size %lld for instance %d", (long long)n_sites, idx);
    if (!dev_state || reinterpret_cast<uintptr_t>(dev_state) % 256)
        return fail(KSLB_EINVAL, "state memory missing or not 256-byte aligned");
    const size_t need = kslb_instance_bytes(n_sites, E->q[idx], E->prec[idx]);
    if (bytes < need) return fail(KSLB_ENOMEM, "instance %d needs %zu bytes, got %zu", idx, need, bytes);
    E->addr[idx] = reinterpret_cast<uintptr_t>(dev_state);
    E->copy[idx] = state_copy_bytes(n_sites, E->q[idx], E->prec[idx]);
    E->cap[idx] = n_sites;
    E->n[idx] = n_sites;
    E->cur[idx] = 0;
    E->have_state[idx] = 0;
    E->step[idx] = 0;
    E->layout_gen++;
    return KSLB_OK;
}

kslb_status kslb_ensemble_init_rho(kslb_ensemble* E, int idx, const double* rho, int on_device)
{
    if (auto s = check_ens(E, idx)) return s;
    if (!rho) return fail(KSLB_EINVAL, "rho must not be NULL");
    if (E->cls[idx] < 0) return fail(KSLB_ESTATE, "set the coefficients of instance %d before init_rho", idx);
    DeviceGuard g(E->device);
    const double* src = rho;
    if (!on_device) {
        if (auto s = ens_staging(E, E->n[idx])) return s;
        int e = hipMemcpyAsync(E->staging, rho, sizeof(double) * (size_t)E->n[idx], hipMemcpyHostToDevice, E->stream);
        if (e) return hip_fail(e, "hipMemcpyAsync(rho)");
        src = E->staging;
    }
    E->cur[idx] = 0;
    int e = launch_init(E->q[idx], E->prec[idx], ens_state(E, idx), E->n[idx], src, E->sets[E->cls[idx]].cf, E->stream);
    if (e) return hip_fail(e, "init kernel");
    if (!on_device) {
        e = hipStreamSynchronize(E->stream);
        if (e) return hip_fail(e, "hipStreamSynchronize");
    }
    E->have_state[idx] = 1;
    E->step[idx] = 0;
    return KSLB_OK;
}

kslb_status kslb_ensemble_init_rho_all(kslb_ensemble* E, const double* rho, int on_device)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    if (!rho) return fail(KSLB_EINVAL, "rho must not be NULL");
    for (int i = 0; i < E->count; i++)
        if (E->cls[i] < 0) return fail(KSLB_ESTATE, "set the coefficients of instance %d before init", i);
    DeviceGuard g(E->device);
    int64_t total = 0;
    std::vector<InstGroup> groups;
    const std::vector<InstDesc> dv = ens_inst_table(E, [](int) { return 0; }, &total, &groups);
    // one upload: the instance table, then the coefficient sets
    const size_t coef_at = sizeof(InstDesc) * dv.size();
    std::vector<char> blob(coef_at + sizeof(Coef) * E->sets.size());
    std::memcpy(blob.data(), dv.data(), coef_at);
    for (size_t j = 0; j < E->sets.size(); j++)
        std::memcpy(blob.data() + coef_at + j * sizeof(Coef), &E->sets[j].cf, sizeof(Coef));
    const double* src = rho;
    if (!on_device) {
        if (auto st = ens_staging(E, total)) return st;
        int e = hipMemcpyAsync(E->staging, rho, sizeof(double) * (size_t)total, hipMemcpyHostToDevice, E->stream);
        if (e) return hip_fail(e, "hipMemcpyAsync(rho)");
        src = E->staging;
    }
    char* dev = nullptr;
    if (auto st = ens_upload(E, E->init_tab, blob.data(), blob.size(), &dev)) return st;
    const InstDesc* dd = reinterpret_cast<const InstDesc*>(dev);
    const Coef* dc = reinterpret_cast<const Coef*>(dev + coef_at);
    for (const InstGroup& gr : groups) {
        int e = launch_init_many(gr.q, gr.prec, dd + gr.begin, gr.end - gr.begin, gr.max_n, dc, src, E->stream);
        if (e) return hip_fail(e, "init kernel");
    }
    if (!on_device) {
        int e = hipStreamSynchronize(E->stream);
        if (e) return hip_fail(e, "hipStreamSynchronize");
    }
    for (int i = 0; i < E->count; i++) {
        E->cur[i] = 0;
        E->have_state[i] = 1;
        E->step[i] = 0;
    }
    return KSLB_OK;
}

kslb_status kslb_ensemble_advance(kslb_ensemble* E, const int64_t* steps)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    if (!steps) return fail(KSLB_EINVAL, "steps must not be NULL");
    for (int i = 0; i < E->count; i++) {
        if (steps[i] < 0) return fail(KSLB_EINVAL, "negative step count for instance %d", i);
        if (steps[i] > 0 && !E->have_state[i]) return fail(KSLB_ESTATE, "instance %d has no state", i);
    }
    DeviceGuard g(E->device);
    std::vector<int64_t> left(steps, steps + E->count);
    std::vector<int> adv(E->count);
    for (;;) {
        bool any = false;
        for (int i = 0; i < E->count; i++) {
            adv[i] = (int)std::min<int64_t>(E->chunk, left[i]);
            any = any || adv[i] > 0;
        }
        if (!any) break;
        if (E->use_graphs) {
            int64_t full = INT64_MAX;
            for (int i = 0; i < E->count; i++) {
                if (left[i] <= 0) continue;
                full = std::min<int64_t>(full, left[i] / E->chunk);
            }
            const int64_t pairs = full / 2;
            if (full != INT64_MAX && pairs >= 2) {
                if (auto s = ens_replay_pairs(E, adv, pairs)) return s;
                for (int i = 0; i < E->count; i++) {
                    if (left[i] <= 0) continue;
                    left[i] -= 2 * pairs * E->chunk;
                    E->step[i] += 2 * pairs * E->chunk;
                }
                continue;
            }
        }
        EnsPlan plan;
        if (auto s = ens_plan(E, adv, &plan)) return s;
        int e = ens_launch(E, plan, E->stream);
        if (e) return hip_fail(e, "ensemble kernel");
        for (int i = 0; i < E->count; i++) {
            if (adv[i] <= 0) continue;
            left[i] -= adv[i];
            E->step[i] += adv[i];
            E->cur[i] ^= 1;
        }
    }
    return KSLB_OK;
}

kslb_status kslb_ensemble_read_rho(kslb_ensemble* E, int idx, double* out, int on_device)
{
    if (auto s = check_ens(E, idx)) return s;
    if (!out) return fail(KSLB_EINVAL, "out must not be NULL");
    if (!E->have_state[idx]) return fail(KSLB_ESTATE, "instance %d has no state", idx);
    DeviceGuard g(E->device);
    double* dst = out;
    if (!on_device) {
        if (auto s = ens_staging(E, E->n[idx])) return s;
        dst = E->staging;
    }
    int e = launch_read_rho(E->q[idx], E->prec[idx], ens_state(E, idx), E->n[idx], dst, E->stream);
    if (e) return hip_fail(e, "readout kernel");
    if (!on_device) {
        e = hipMemcpyAsync(out, dst, sizeof(double) * (size_t)E->n[idx], hipMemcpyDeviceToHost, E->stream);
        if (!e) e = hipStreamSynchronize(E->stream);
        if (e) return hip_fail(e, "readout copy");
    }
    return KSLB_OK;
}

kslb_status kslb_ensemble_read_rho_all(kslb_ensemble* E, double* out, int on_device)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    if (!out) return fail(KSLB_EINVAL, "out must not be NULL");
    for (int i = 0; i < E->count; i++)
        if (!E->have_state[i]) return fail(KSLB_ESTATE, "instance %d has no state", i);
    DeviceGuard g(E->device);
    int64_t total = 0;
    std::vector<InstGroup> groups;
    const std::vector<InstDesc> dv = ens_inst_table(E, [&](int i) { return E->cur[i]; }, &total, &groups);
    double* dst = out;
    if (!on_device) {
        if (auto st = ens_staging(E, total)) return st;
        dst = E->staging;
    }
    char* dev = nullptr;
    if (auto st = ens_upload(E, E->read_tab, dv.data(), sizeof(InstDesc) * dv.size(), &dev)) return st;
    const InstDesc* dd = reinterpret_cast<const InstDesc*>(dev);
    for (const InstGroup& gr : groups) {
        int e = launch_read_many(gr.q, gr.prec, dd + gr.begin, gr.end - gr.begin, gr.max_n, dst, E->stream);
        if (e) return hip_fail(e, "readout kernel");
    }
    if (!on_device) {
        int e = hipMemcpyAsync(out, dst, sizeof(double) * (size_t)total, hipMemcpyDeviceToHost, E->stream);
        if (!e) e = hipStreamSynchronize(E->stream);
        if (e) return hip_fail(e, "readout copy");
    }
    return KSLB_OK;
}

kslb_status kslb_ensemble_status(kslb_ensemble* E, int idx, int64_t* step, int* nonfinite)
{
    if (auto s = check_ens(E, idx)) return s;
    if (step) *step = E->step[idx];
    if (!nonfinite) return KSLB_OK;
    if (!E->have_state[idx]) { *nonfinite = 0; return KSLB_OK; }
    DeviceGuard g(E->device);
    double* partial = reinterpret_cast<double*>(E->buf + E->diag_off);
    double* mass_d = partial + 256;
    int* flag_d = reinterpret_cast<int*>(partial + 257);
    int e = launch_diag(E->q[idx], E->prec[idx], ens_state(E, idx), E->n[idx], partial, flag_d, mass_d, E->stream);
    if (e) return hip_fail(e, "diagnostics kernel");
    int f = 0;
    e = hipMemcpyAsync(&f, flag_d, sizeof f, hipMemcpyDeviceToHost, E->stream);
    if (!e) e = hipStreamSynchronize(E->stream);
    if (e) return hip_fail(e, "diagnostics copy");
    *nonfinite = f;
    return KSLB_OK;
}

kslb_status kslb_ensemble_renormalize(kslb_ensemble* E, int npairs, const int* ref, const int* pert, double delta,
                                      double* log_accum)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    if (npairs < 0 || (npairs > 0 && (!ref || !pert || !log_accum)))
        return fail(KSLB_EINVAL, "bad pair arguments");
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(KSLB_EINVAL, "delta must be positive and finite");
    if (npairs == 0) return KSLB_OK;
    std::vector<PairDesc> pd((size_t)npairs);
    int nq5 = 0;   // pairs of D1Q5 instances, placed first in the table
    for (int p = 0; p < npairs; p++) {
        const int a = ref[p], b = pert[p];
        if (a < 0 || a >= E->count || b < 0 || b >= E->count || a == b)
            return fail(KSLB_EINVAL, "pair %d: bad instances (%d, %d)", p, a, b);
        if (E->prec[a] != kFP64 || E->prec[b] != kFP64)
            return fail(KSLB_EINVAL, "pair %d: trajectory pairs need FP64 storage", p);
        if (E->q[a] != E->q[b]) return fail(KSLB_EINVAL, "pair %d: instances differ in scheme", p);
        if (!E->have_state[a] || !E->have_state[b]) return fail(KSLB_ESTATE, "pair %d: instance without state", p);
        if (E->n[a] != E->n[b] || E->step[a] != E->step[b])
            return fail(KSLB_EINVAL, "pair %d: instances differ in sites or steps", p);
        nq5 += E->q[a] == 5;
    }
    for (int p = 0; p < npairs; p++)
        for (int r = p + 1; r < npairs; r++)
            if (pert[p] == pert[r] || pert[p] == ref[r] || ref[p] == pert[r])
                return fail(KSLB_EINVAL, "pairs %d and %d share a perturbed instance", p, r);
    int at5 = 0, at7 = nq5;
    for (int p = 0; p < npairs; p++) {
        const int a = ref[p], b = pert[p];
        pd[E->q[a] == 5 ? at5++ : at7++] =
            PairDesc{ens_addr(E, a, E->cur[a]), ens_addr(E, b, E->cur[b]), E->n[a], state_pitch(E->n[a]), p, 0};
    }
    DeviceGuard g(E->device);
    const size_t bytes = sizeof(PairDesc) * (size_t)npairs;
    int e = 0;
    if (E->pairs_pending) {   // the staging may still feed the previous upload
        e = hipEventSynchronize(E->pairs_ev);
        if (e) return hip_fail(e, "pair table event");
        E->pairs_pending = false;
    }
    if (E->pairs_cap < bytes) {
        if (E->d_pairs) (void)hipFree(E->d_pairs);
        if (E->h_pairs) (void)hipHostFree(E->h_pairs);
        E->d_pairs = E->h_pairs = nullptr;
        E->pairs_cap = 0;
        void* dp = nullptr;
        void* hp = nullptr;
        if (hipMalloc(&dp, bytes)) return fail(KSLB_ENOMEM, "pair table of %zu bytes", bytes);
        if (hipHostMalloc(&hp, bytes, hipHostMallocDefault)) {
            (void)hipFree(dp);
            return fail(KSLB_ENOMEM, "pinned pair table of %zu bytes", bytes);
        }
        E->d_pairs = (char*)dp;
        E->h_pairs = (char*)hp;
        E->pairs_cap = bytes;
    }
    if (!E->pairs_ev && hipEventCreateWithFlags(&E->pairs_ev, hipEventDisableTiming))
        return fail(KSLB_EDEVICE, "event creation failed");
    std::memcpy(E->h_pairs, pd.data(), bytes);
    e = hipMemcpyAsync(E->d_pairs, E->h_pairs, bytes, hipMemcpyHostToDevice, E->stream);
    if (!e) e = hipEventRecord(E->pairs_ev, E->stream);
    if (e) return hip_fail(e, "pair table upload");
    E->pairs_pending = true;
    const PairDesc* dt = reinterpret_cast<const PairDesc*>(E->d_pairs);
    if (nq5) e = launch_pair_renorm(5, dt, nq5, delta, log_accum, E->stream);
    if (!e && npairs > nq5) e = launch_pair_renorm(7, dt + nq5, npairs - nq5, delta, log_accum, E->stream);
    if (e) return hip_fail(e, "pair renormalisation kernel");
    return KSLB_OK;
}

kslb_status kslb_ensemble_orthonormalize(kslb_ensemble* E, int ngroups, int k, const int* ref, const int* pert,
                                         double delta, double* log_accum)
{
    if (!E) return fail(KSLB_EINVAL, "null ensemble");
    if (ngroups < 0 || k < 1 || k > kGroupMaxK || (ngroups > 0 && (!ref || !pert || !log_accum)))
        return fail(KSLB_EINVAL, "bad group arguments (1 <= k <= %d)", kGroupMaxK);
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(KSLB_EINVAL, "delta must be positive and finite");
    if (ngroups == 0) return KSLB_OK;
    std::vector<char> used((size_t)E->count, 0);
    int nq5 = 0;
    for (int g = 0; g < ngroups; g++) {
        const int a = ref[g];
        for (int m = -1; m < k; m++) {
            const int i = m < 0 ? a : pert[(size_t)g * k + m];
            if (i < 0 || i >= E->count) return fail(KSLB_EINVAL, "group %d: instance %d out of range", g, i);
            if (used[i]) return fail(KSLB_EINVAL, "group %d: instance %d appears twice", g, i);
            used[i] = 1;
            if (E->prec[i] != kFP64) return fail(KSLB_EINVAL, "group %d: trajectories need FP64 storage", g);
            if (!E->have_state[i]) return fail(KSLB_ESTATE, "group %d: instance %d has no state", g, i);
            if (E->q[i] != E->q[a] || E->n[i] != E->n[a] || E->step[i] != E->step[a])
                return fail(KSLB_EINVAL, "group %d: instances differ in scheme, sites or steps", g);
        }
        nq5 += E->q[a] == 5;
    }
    // table: group descriptors (D1Q5 groups first), then the perturbed-state addresses
    std::vector<GroupDesc> gv((size_t)ngroups);
    std::vector<uint64_t> offs((size_t)ngroups * k);
    int at5 = 0, at7 = nq5;
    for (int g = 0; g < ngroups; g++) {
        const int a = ref[g];
        const int row = E->q[a] == 5 ? at5++ : at7++;
        gv[row] = GroupDesc{ens_addr(E, a, E->cur[a]), E->n[a], state_pitch(E->n[a]),
                            row * k, k, g * k, 0};
        for (int m = 0; m < k; m++) {
            const int i = pert[(size_t)g * k + m];
            offs[(size_t)row * k + m] = ens_addr(E, i, E->cur[i]);
        }
    }
    const size_t off_at = sizeof(GroupDesc) * gv.size();
    std::vector<char> blob(off_at + sizeof(uint64_t) * offs.size());
    std::memcpy(blob.data(), gv.data(), off_at);
    std::memcpy(blob.data() + off_at, offs.data(), sizeof(uint64_t) * offs.size());
    DeviceGuard dg(E->device);
    char* dev = nullptr;
    if (auto st = ens_upload(E, E->group_tab, blob.data(), blob.size(), &dev)) return st;
    const GroupDesc* dd = reinterpret_cast<const GroupDesc*>(dev);
    const uint64_t* doff = reinterpret_cast<const uint64_t*>(dev + off_at);
    int e = 0;
    if (nq5) e = launch_group_orth(5, k, dd, doff, nq5, delta, log_accum, E->stream);
    if (!e && ngroups > nq5) e = launch_group_orth(7, k, dd + nq5, doff, ngroups - nq5, delta, log_accum, E->stream);
    if (e) return hip_fail(e, "group orthonormalisation kernel");
    return KSLB_OK;
}

kslb_status kslb_ensemble_destroy(kslb_ensemble* E)
{
    if (!E) return KSLB_OK;
    DeviceGuard g(E->device);
    (void)hipStreamSynchronize(E->stream);
    if (E->gexec) (void)hipGraphExecDestroy(E->gexec);
    ens_reap_graphs(E, true);
    if (E->cap_stream) (void)hipStreamDestroy(E->cap_stream);
    for (int k = 0; k < 2; k++) {
        if (E->d_tab[k]) (void)hipFree(E->d_tab[k]);
        if (E->h_pin[k]) (void)hipHostFree(E->h_pin[k]);
        if (E->up_ev[k]) (void)hipEventDestroy(E->up_ev[k]);
    }
    if (E->staging) (void)hipFree(E->staging);
    if (E->d_pairs) (void)hipFree(E->d_pairs);
    if (E->h_pairs) (void)hipHostFree(E->h_pairs);
    if (E->pairs_ev) (void)hipEventDestroy(E->pairs_ev);
    ens_table_free(E->init_tab);
    ens_table_free(E->read_tab);
    ens_table_free(E->group_tab);
    delete E;
    return KSLB_OK;
}

}  // extern "C"
