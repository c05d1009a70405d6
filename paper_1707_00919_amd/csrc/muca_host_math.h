// muca_host_math.h -- host arithmetic of libmuca that needs no device (see
// muca_host_math.cpp).  Not part of the public C ABI; plain C++, no HIP.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace muca_host {

// Acceptance thresholds T[k*5+d] from the log weights (IEEE double, libm exp).
void compute_thresholds(uint32_t N, const double* om, uint64_t* t5);
// Generic-kernel table: uint64 thresholds of the four energy-changing moves.
void device_table(uint32_t N, const uint64_t* t5, uint64_t* t4);
// Table of the fast, split and wide kernels: uint32 S = T - 1 at f[k*stride + m]
// by the number m of anti-aligned neighbours (stride 5, or 8 for the wide
// kernel's 32-byte records, the rest zero); false if a move that can be
// proposed has T = 0.
bool fast_table(uint32_t N, const uint64_t* t5, uint32_t* f, uint32_t stride);
double flatness_of(uint32_t N, const uint64_t* H);
double chebyshev_of(uint32_t N, const uint64_t* H);
// ln g[k] = ln H[k] - omega[k] + c on reachable bins with H > 0, -inf
// elsewhere; normalization 0: ln g[0] = ln 2, 1: sum exp(ln g) = 2^N.
// Returns 0, or 1 (ground-state bin empty) / 2 (histogram empty).
int log_dos_of(uint32_t N, const uint64_t* H, const double* omega, int normalization, double* out);
// Eq. 6 with Q uniform over max(reach_prev, 10) bins.
double kl_of(uint32_t N, const uint64_t* H, int reach_prev);
// Reachable bins (not 1 or N-1) between the lowest and highest visited bin.
int reach_of(uint32_t N, const uint64_t* H);
int width_of(uint32_t N, const uint64_t* H);

// One piece of a call: whole sweeps [sweep0, sweep0 + n) of which the first
// `therm` are not recorded, or (n == 0) the sites [site_begin, site_end) of
// sweep sweep0 with recording from site rec_begin on.
struct Segment {
    uint64_t sweep0;
    uint64_t n;
    uint64_t therm;
    uint32_t site_begin, site_end, rec_begin;
};

// Cuts the attempts [pos0, pos0 + therm + recorded) -- recording from
// pos0 + therm on -- into whole-sweep runs for the sweep kernels and partial
// sweeps for the range kernel.
std::vector<Segment> segments_of(uint64_t N, uint64_t pos0, uint64_t therm, uint64_t recorded);

}  // namespace muca_host
