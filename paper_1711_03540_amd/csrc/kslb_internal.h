// kslb_internal.h -- declarations shared by the host parameter code, the HIP
// kernels and the C ABI of libkslb.  Not installed; not part of the ABI.
#pragma once

#include <cstddef>
#include <cstdint>

namespace kslb {

// tau below this is refused: M of Table 2 has a pole where T4 + 1 = 0
// (tau = (3 + sqrt 6)/6 ~ 0.908).
constexpr double kTauMin = 0.92;

enum Precision { kFP64 = 0, kFP32 = 1, kSPLIT = 2, kRHO = 3 };

// Coefficients handed to every kernel by value.
//   feq_i(rho) = E_i rho + G_i rho^2        (equilibrium, section 2.3)
//   A_i = omega E_i,  B_i = omega G_i,  a1mw = 1 - omega
// so the BGK collision of Eq. (2) is  f'_i = a1mw f_i + A_i rho + B_i rho^2.
struct Coef {
    double E[7];
    double G[7];
    double A[7];
    double B[7];
    double a1mw;
    float a1mw_f;
    float pad_;
};

// host parameter code (kslb_params.cpp)
void scheme_weights(int q, double w[7][7]);
int scheme_coefficients(int q, double dX, double dT, double tau, int dm_variant, double jkm[5],
                        double* E, double* G);
double tau_fit(int q, double dX, double dT);
double spectral_radius(int q, const double* E, const double* G, double omega, double rho_bar,
                       double k);
int stability_check(int q, const double* E, const double* G, double omega, double dX, double dT,
                    double rho_max);

// row pitch (sites) and bytes of one copy of the state of n sites
int64_t state_pitch(int64_t n);
size_t state_copy_bytes(int64_t n, int q, int prec);

// ---------------------------------------------------------------------------
// kernel launchers (kslb_kernels.hip).  All return a hipError_t as int.
// ---------------------------------------------------------------------------
// lanes and LDS bytes of the ring (one workgroup per lattice) and tile kernels
int ring_max_lanes();
int tile_lanes();
int ring_lds_bytes(int q);
int tile_lds_bytes(int q);
int max_lds_bytes();

int launch_init(int q, int prec, void* state, int64_t n, const double* rho0, const Coef& cf,
                void* stream);
int launch_plain(int q, int prec, const void* src, void* dst, int64_t n, const Coef& cf,
                 void* stream);
int launch_ring(int q, int prec, int B, const void* src, void* dst, int64_t n, int64_t steps,
                const Coef& cf, void* stream);
// rho0 / rho_out (16-byte aligned, may be null): start from feq(rho0)
// instead of src, and write the density of every site as well as dst.
int launch_tile(int q, int prec, const void* src, void* dst, int64_t n, int s,
                const Coef& cf, void* stream, const double* rho0 = nullptr, double* rho_out = nullptr);
// Sites per lane of the tiled kernel for a storage mode (its window holds
// tile_lanes() * that many sites).
int tile_sites_per_lane(int prec);
// One small lattice over nwg single-wave workgroups exchanging edges every s
// steps through `slots` edge slots per launch (slots * nwg copies of ecopy
// bytes from ebase, each holding one owner's own sites in state format; see
// span_edge_copy_bytes).  ctl holds
// span_ctl_ints() ints (abort word, sticky error word, abort claim, count of
// aborted launches), set up by launch_span_ctl_init.  The state is read from
// src and written to dst.
int span_lanes();
int span_sites_per_lane(int q, int prec);
int span_ctl_ints();
int span_ctl_error_index();   // sticky: a launch stopped early since the state was set
int span_ctl_aborts_index();  // launches that stopped early since the control block was set up
// owners of this kernel variant the current device keeps resident (0 if unknown)
int64_t span_device_owners(int q, int prec, bool fixed);
// Static edge-slot area of the no-allocation advance, and its device address
// on the current device (looked up on a device's first call).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
int noalloc_scratch(char** ptr);
int64_t span_edge_copy_bytes(int q, int prec, int64_t n, int nwg, int s);   // one slot copy
int launch_span_ctl_init(int* ctl, int count, void* stream);
int launch_span_set_ctl(int* ctl, int index, int value, void* stream);
// Trajectory pair of an FP64 ensemble: device addresses of the two current
// state copies, sites, row pitch and the accumulator slot.
struct PairDesc {
    uint64_t ref, pert;
    int64_t n, pitch;
    int32_t slot, pad;
};
int launch_pair_renorm(int q, const PairDesc* desc, int npairs, double delta, double* log_accum, void* stream);
// A reference and k perturbed copies of an FP64 ensemble: device address of
// the reference's current state copy, sites, row pitch, the index of the
// group's first perturbed-state address in a separate array, k, and the first
// of its k accumulator slots.
constexpr int kGroupMaxK = 8;
struct GroupDesc {
    uint64_t ref;
    int64_t n, pitch;
    int32_t first, k, slot, pad;
};
int launch_group_orth(int q, int k, const GroupDesc* desc, const uint64_t* pert, int ngroups, double delta,
                      double* log_accum, void* stream);
// fixed-end boundary values (NULL / absent = periodic)
struct Ends {
    double rho_l, rho_r;
};
// inject_abort: start with the abort word raised (every owner stops at its
// first exchange and the sticky error word is set), for failure-path tests.
int launch_span(int q, int prec, const void* src, void* dst, int64_t n, int nwg, int64_t steps, int s, char* ebase,
                int64_t ecopy, int64_t slots, int* ctl, const Coef& cf, void* stream, const Ends* ends,
                bool inject_abort = false);
int launch_plain_fixed(int q, int prec, const void* src, void* dst, int64_t n, const Coef& cf, const Ends& ends,
                       void* stream);
int launch_init_fixed(int q, int prec, void* state, int64_t n, const double* rho0, const Coef& cf, const Ends& ends,
                      void* stream);
// err: the lattice's sticky error word (or null); while it is set the
// readouts write NaN
int launch_read_rho(int q, int prec, const void* state, int64_t n, double* out, void* stream,
                    const int* err = nullptr);
int launch_read_f(int q, int prec, const void* state, int64_t n, double* out, int pre,
                  const Coef& cf, void* stream, const int* err = nullptr);
int launch_write_f(int q, int prec, void* state, int64_t n, const double* in, const Coef& cf,
                   void* stream);
int launch_diag(int q, int prec, const void* state, int64_t n, double* partial, int* flag,
                double* mass_out, void* stream);

// ensemble: one window per workgroup; a window holds one or more segments,
// each a tile of one instance on a consecutive range of lanes.  Every
// segment of a window shares the window's step count and coefficient set.
struct WinHdr {
    int32_t first_seg;  // index of the window's first segment
    int32_t nseg;       // segments in the window (>= 1)
    int32_t steps;      // steps every segment of the window advances
    int32_t coef;       // index of the window's coefficient set in the launch's table
};
struct SegDesc {
    uint64_t src;       // device address of the instance's source state copy
    uint64_t dst;       // device address of the destination state copy
    int64_t n;          // sites of the instance
    int64_t pitch;      // row pitch of the instance (state_pitch(n))
    int64_t start;      // site of the segment's first slot (may be negative: periodic)
    int32_t lane_lo;    // first lane of the segment
    int32_t valid;      // sites written back, from slot H * steps on
};
// One ensemble instance in a batched init or readout: device address of its
// state copy, offset of its densities in the packed density array, sites,
// row pitch and coefficient set (init only).
struct InstDesc {
    uint64_t state;
    int64_t rho_off, n, pitch;
    int32_t coef, pad;
};
// Instances desc[0 .. count) of one scheme and storage; max_n bounds their sizes.
int launch_init_many(int q, int prec, const InstDesc* desc, int count, int64_t max_n, const Coef* coefs,
                     const double* rho, void* stream);
int launch_read_many(int q, int prec, const InstDesc* desc, int count, int64_t max_n, double* rho, void* stream);

// coefs: device table of coefficient sets, indexed by WinHdr::coef
int launch_ens(int q, int prec, int B, const WinHdr* hdr, const SegDesc* seg, int nwin,
               const Coef* coefs, void* stream);

}  // namespace kslb
