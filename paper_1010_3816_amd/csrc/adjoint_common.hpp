// Pieces shared by the adjoint-side kernels (adjoint_kernels.hip) and the
// forward-mode spin derivative (spin_tangent.hip): LDS views of the radial
// tables, the a-derivatives of the coefficients, and the strip-major tiles
// of a workgroup.
#pragma once

#include "device_common.hpp"

namespace teuk {
namespace {

// LDS copy of a strip's radial tables: [value/derivative][integer/half][field][lane].
// `o` is a row-dependent offset that is 0 at run time (row & zero): it keeps
// the reads inside the row loop instead of in (scarce) registers.
typedef const __attribute__((address_space(3))) double* lds_cptr;

__device__ __forceinline__ Rad rad_from_lds(lds_cptr rs, int o) {
    Rad R;
    R.rho = rs[o + R_RHO * kWave];
    R.rho2 = rs[o + R_RHO2 * kWave];
    R.a2d = rs[o + R_A2D * kWave];
    R.rb1 = rs[o + R_RB1 * kWave];
    R.rb2 = rs[o + R_RB2 * kWave];
    R.rb3 = rs[o + R_RB3 * kWave];
    R.ctr = rs[o + R_CTR * kWave];
    R.cti0 = rs[o + R_CTI0 * kWave];
    R.cti1 = rs[o + R_CTI1 * kWave];
    R.b1n = rs[o + R_B1N * kWave];
    R.dl2 = rs[o + R_DL2 * kWave];
    R.v0r = rs[o + R_V0R * kWave];
    R.v0i = rs[o + R_V0I * kWave];
    return R;
}

// d/da of kerr_coef at one position from the radial factors V and their
// a-derivatives D (as kerr_coef_da).
__device__ __forceinline__ Coef kerr_coef_da_reg(const Rad& V, const Rad& D, const Ang& G, Sig s, const Coef& c) {
    const double w = s.inv * fma(-D.a2d, G.sn2, D.rho2);
    const double hw = 0.5 * w;
    Coef r;
    r.b = fma(s.isig, D.rho, -c.b * hw);
    const double T = fma(-V.rb3, G.sn2, V.rb2);
    const double dT = fma(-D.rb3, G.sn2, D.rb2);
    const double Q = fma(-T, s.inv, V.rb1);
    const double dQ = fma(-s.inv, fma(-T, w, dT), D.rb1);
    const double bp = s.isig * Q;
    const double dbp = s.isig * fma(-Q, hw, dQ);
    r.ctr = fma(s.inv, D.ctr, -c.ctr * w);
    r.cti = fma(s.inv, fma(D.cti1, G.cs, D.cti0), -c.cti * w);
    const double b1 = V.b1n * s.inv;
    const double db1 = fma(s.inv, D.b1n, -b1 * w);
    r.cre = fma(r.b, bp - c.ctr, c.b * (dbp - r.ctr)) - db1;
    r.cim = -fma(r.b, c.cti, c.b * r.cti);
    r.a2s = fma(s.inv, D.dl2, -c.a2s * w);
    r.a1s = r.a2s * G.cotp;
    r.v0r = fma(s.inv, fma(D.dl2, G.pd, D.v0r), -c.v0r * w);
    r.v0i = fma(s.inv, D.v0i, -c.v0i * w);
    return r;
}

// Tile of a wavefront.  Tiles are numbered strip-major (the theta chunks of
// a strip consecutive) and workgroup b takes tiles b*wpb .. b*wpb + wpb - 1,
// so the tile count need not be a multiple of wpb per strip and a launch can
// fill every wavefront slot of the device.  A workgroup's tiles lie in at
// most two consecutive strips when wpb <= n_chunks + 1 (the host keeps it
// so); it holds the radial tables of both in LDS, as two slices.
struct TileOf {
    int strip, chunk;  // of this wavefront's tile
    int s0, n_slices;  // the workgroup's first strip and its number of strips (1 or 2)
    int slice;         // this wavefront's slice, strip - s0
    bool valid;        // false for wavefronts past the last tile
};

__device__ __forceinline__ TileOf tile_of(int b, int wpb, int wave, int n_strips, int n_chunks) {
    TileOf T;
    const int n_tiles = n_strips * n_chunks;
    const int first = b * wpb, tile = first + wave;
    T.valid = tile < n_tiles;
    T.s0 = first / n_chunks;
    T.n_slices = min((min(first + wpb, n_tiles) - 1) / n_chunks - T.s0 + 1, 2);
    T.strip = min(tile, n_tiles - 1) / n_chunks;
    T.chunk = tile - T.strip * n_chunks;
    T.slice = min(T.strip - T.s0, 1);
    return T;
}

// Workgroups of wpb consecutive tiles (strip-major), wpb at most n_chunks + 1
// so that a workgroup spans at most two strips.  The LDS holds one strip's
// tables (fields_per_strip doubles per lane) when no workgroup spans two,
// i.e. when wpb divides the chunks of a strip or there is one strip, and two
// otherwise.
inline void adjoint_launch_shape(const AdjScalars& k, int waves_per_block, int fields_per_strip, dim3* grid,
                                 dim3* block, size_t* lds_bytes) {
    const int w = std::min(waves_per_block, k.n_chunks + 1);
    const int64_t tiles = (int64_t)k.n_strips * k.n_chunks;
    const int slices = (k.n_chunks % w == 0 || k.n_strips == 1) ? 1 : 2;
    *block = dim3(kWave * w);
    *grid = dim3((unsigned)((tiles + w - 1) / w));
    *lds_bytes = (size_t)slices * fields_per_strip * kWave * sizeof(double);
}

}  // namespace
}  // namespace teuk
